// Learned preconditioner network for gfx950: a small U-Net (3x3 convolutions,
// 2x2 average pooling, nearest upsampling with skip concatenation, 1x1 head)
// with BF16 MFMA (FP32 accumulate) forward, input-gradient and weight-gradient
// kernels, and Adam on FP32 master weights.  The convolutions run on gfx950's
// v_mfma_f32_16x16x32_bf16 with the input tile and the weights staged in LDS
// (k_conv3t); the K = 16 kernel (v_mfma_f32_16x16x16_bf16) remains for the weight
// gradient and as the fallback of the convolution (inputs of other than a multiple
// of 16 channels: the first layer).
//
// Activations are NHWC.  A 3x3 convolution is an implicit GEMM: M = pixels,
// N = output channels, K = 9 taps x input channels (in chunks of 16).  The input
// gradient is the same kernel run on the output gradient with the weights flipped
// in both spatial directions and transposed in channels.  The weight gradient is a
// GEMM over pixels (K = pixels) on channel-major copies, split over pixel chunks
// and reduced in a fixed order.
//
// MFMA 16x16x16 operand layout (lane l, element r = 0..3):
//   A[i][k]: i = l % 16, k = 4 (l / 16) + r;  B[k][j]: j = l % 16, k = 4 (l / 16) + r;
//   D[i][j]: j = l % 16, i = 4 (l / 16) + r.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/m1.h"
#include "m1_internal.h"
#include "m1_nn.h"

namespace m1 {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x4 load4(const uint16_t* p) {
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  bf16x4 r;
  r[0] = (short)(v.x & 0xFFFF);
  r[1] = (short)(v.x >> 16);
  r[2] = (short)(v.y & 0xFFFF);
  r[3] = (short)(v.y >> 16);
  return r;
}
__device__ __forceinline__ bf16x4 load4(const float* p) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  bf16x4 r;
  r[0] = (short)f2bf(v.x);
  r[1] = (short)f2bf(v.y);
  r[2] = (short)f2bf(v.z);
  r[3] = (short)f2bf(v.w);
  return r;
}
__device__ __forceinline__ void store1(uint16_t* p, float v) { *p = f2bf(v); }
__device__ __forceinline__ void store1(float* p, float v) { *p = v; }

// ---------------------------------------------------------------------------
// 3x3 convolution (forward, or input gradient with transformed weights)
// Input channels: [0, C0) from x0 (optionally at half resolution, nearest
// upsampled), [C0, C0 + C1) from x1.  w: [9][Cout][C0 + C1] bf16.
// Block: 4 wavefronts x 16 pixels of one row; each wave covers 64 output channels.
// ---------------------------------------------------------------------------
template <typename TIN, typename TOUT>
__global__ __launch_bounds__(256) void k_conv3(int H, int W, const TIN* __restrict__ x0, int C0, int up0,
                                               const TIN* __restrict__ x1, int C1, const uint16_t* __restrict__ w,
                                               const float* __restrict__ bias, int Cout, TOUT* __restrict__ y,
                                               int relu, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int h = blockIdx.y;
  const int pbase = blockIdx.x * 64 + wv * 16;
  if (pbase >= W) return;  // whole wavefront idle
  const int co_base = blockIdx.z * 64;
  const int pA = pbase + (lane & 15);
  const int kq = (lane >> 4) * 4;
  const int Cin = C0 + C1;
  const int W0 = up0 ? (W >> 1) : W;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x4 zero = {0, 0, 0, 0};
  for (int tap = 0; tap < 9; ++tap) {
    const int hh = h + tap / 3 - 1, ww = pA + tap % 3 - 1;
    const bool inb = hh >= 0 && hh < H && ww >= 0 && ww < W;
    for (int c0 = 0; c0 < Cin; c0 += 16) {
      bf16x4 A = zero;
      if (inb) {
        if (c0 < C0) {
          const int sh = up0 ? (hh >> 1) : hh, sw = up0 ? (ww >> 1) : ww;
          A = load4(x0 + ((int64_t)sh * W0 + sw) * C0 + c0 + kq);
        } else {
          A = load4(x1 + ((int64_t)hh * W + ww) * C1 + (c0 - C0) + kq);
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int co = co_base + t * 16 + (lane & 15);
        const bf16x4 B = co < Cout ? load4(w + ((int64_t)tap * Cout + co) * Cin + c0 + kq) : zero;
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc[t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int co = co_base + t * 16 + (lane & 15);
    if (co >= Cout) continue;
    const float b = bias ? bias[co] : 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int px = pbase + (lane >> 4) * 4 + r;
      if (px >= W) continue;
      float v = acc[t][r] + b;
      if (relu) v = fmaxf(v, 0.f);
      store1(y + ((int64_t)h * W + px) * Cout + co, v);
    }
  }
}

// ---------------------------------------------------------------------------
// gfx950's K = 32 MFMA (v_mfma_f32_16x16x32_bf16): each lane supplies 8 consecutive
// channels of one pixel (A) and of one output channel's weights (B); the sum over k
// is the same whatever order the hardware pairs the lanes' k slots in, since A and B
// use one convention.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}
__device__ __forceinline__ bf16x8 load8(const float* p) {
  const float4 u = *reinterpret_cast<const float4*>(p);
  const float4 v = *reinterpret_cast<const float4*>(p + 4);
  uint4 r;
  r.x = (uint32_t)f2bf(u.x) | ((uint32_t)f2bf(u.y) << 16);
  r.y = (uint32_t)f2bf(u.z) | ((uint32_t)f2bf(u.w) << 16);
  r.z = (uint32_t)f2bf(v.x) | ((uint32_t)f2bf(v.y) << 16);
  r.w = (uint32_t)f2bf(v.z) | ((uint32_t)f2bf(v.w) << 16);
  return __builtin_bit_cast(bf16x8, r);
}

// ---------------------------------------------------------------------------
// The convolution with the input tile and all nine taps' weights in LDS, one
// 32-channel slice of the input at a time: a block (4 waves) computes 4 RW rows x 64
// pixels x 16 NT output channels.  Per slice it stages the (4 RW + 2) x 66 input
// pixels around the tile and the 9 x 16 NT weight rows, then each wave runs 9 taps x
// RW x 4 x NT MFMAs (16x16x32 bf16, same operand convention as above) from LDS: two barriers
// per 32 input channels, and every input element is read from memory once per
// block (a per-tap form, which staged one tap's weights at a time and read the input
// from memory once per tap, took two barriers per tap and was no faster than the
// K = 16 kernel).  Requires C0 % 8 == 0 and Cin % 16 == 0.
// ---------------------------------------------------------------------------
constexpr int kCT = 32;            // input channels per slice
constexpr int kCTP = kCT + 8;      // padded LDS row (bf16), against bank conflicts
constexpr int kConvRowsPerWave = 1;  // output rows per wavefront (two measured slower: 0.62 against 0.46 ms per pass)

template <int NT, int RW, typename TIN, typename TOUT>
__global__ __launch_bounds__(256) void k_conv3t(int H, int W, const TIN* __restrict__ x0, int C0, int up0,
                                                const TIN* __restrict__ x1, int C1, const uint16_t* __restrict__ w,
                                                const float* __restrict__ bias, int Cout, TOUT* __restrict__ y,
                                                int relu, const int* __restrict__ skip, TOUT* __restrict__ ypool) {
  constexpr int ROWS = 4 * RW;          // output rows of the block (RW per wave)
  constexpr int IR = ROWS + 2;          // input rows staged
  __shared__ __align__(16) uint16_t sx[IR * 66 * kCTP];
  __shared__ __align__(16) uint16_t swt[9 * 16 * NT * kCTP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int h0 = blockIdx.y * ROWS;
  const int pbase = blockIdx.x * 64;
  const int co_base = blockIdx.z * 16 * NT;
  const int Cin = C0 + C1;
  const int W0 = up0 ? (W >> 1) : W;
  const int kq = (lane >> 4) * 8;
  f32x4 acc[RW][4][NT];
#pragma unroll
  for (int q = 0; q < RW; ++q)
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[q][g][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x8 zero = __builtin_bit_cast(bf16x8, make_uint4(0u, 0u, 0u, 0u));
  // staging work per 32-channel slice: input rows h0 - 1 .. h0 + ROWS, pixels pbase - 1 ..
  // pbase + 64 (zero outside the image), four 8-channel groups; the nine taps' weights of
  // the block's output channels, swt[tap][col][ci].  A thread issues all of its loads
  // before it stores any, and the next slice's loads are issued before the current
  // slice's MFMAs, so the slices' memory round trips overlap the arithmetic.
  constexpr int NIN = IR * 66 * 4, NWT = 9 * 16 * NT * 4;
  constexpr int PIN = (NIN + 255) / 256, PWT = (NWT + 255) / 256;
  bf16x8 vin[PIN];
  uint4 vwt[PWT];
  auto load_slice = [&](int c0) {
#pragma unroll
    for (int it = 0; it < PIN; ++it) {
      const int e = threadIdx.x + it * 256;
      const int grp = e & 3, pix = e >> 2;
      const int r = pix / 66, p = pix - r * 66;
      const int hh = h0 - 1 + r, ww = pbase - 1 + p;
      const int k = c0 + grp * 8;
      vin[it] = zero;
      if (e < NIN && k < Cin && hh >= 0 && hh < H && ww >= 0 && ww < W) {
        if (k < C0) {
          const int sh = up0 ? (hh >> 1) : hh, sw0 = up0 ? (ww >> 1) : ww;
          vin[it] = load8(x0 + ((int64_t)sh * W0 + sw0) * C0 + k);
        } else {
          vin[it] = load8(x1 + ((int64_t)hh * W + ww) * C1 + (k - C0));
        }
      }
    }
#pragma unroll
    for (int it = 0; it < PWT; ++it) {
      const int e = threadIdx.x + it * 256;
      const int grp = e & 3, row = e >> 2;
      const int tap = row / (16 * NT), col = row - tap * (16 * NT);
      const int co = co_base + col, k = c0 + grp * 8;
      vwt[it] = make_uint4(0u, 0u, 0u, 0u);
      if (e < NWT && co < Cout && k < Cin) vwt[it] = *reinterpret_cast<const uint4*>(w + ((int64_t)tap * Cout + co) * Cin + k);
    }
  };
  load_slice(0);
  float bv[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int co = co_base + t * 16 + (lane & 15);
    bv[t] = (bias && co < Cout) ? bias[co] : 0.f;
  }
  if (skip && *skip) return;   // the flag is uniform: the whole block leaves
  for (int c0 = 0; c0 < Cin; c0 += kCT) {
    __syncthreads();   // the previous slice is consumed
#pragma unroll
    for (int it = 0; it < PIN; ++it) {
      const int e = threadIdx.x + it * 256;
      if (e < NIN) *reinterpret_cast<bf16x8*>(sx + (e >> 2) * kCTP + (e & 3) * 8) = vin[it];
    }
#pragma unroll
    for (int it = 0; it < PWT; ++it) {
      const int e = threadIdx.x + it * 256;
      if (e < NWT) *reinterpret_cast<uint4*>(swt + (e >> 2) * kCTP + (e & 3) * 8) = vwt[it];
    }
    __syncthreads();
    if (c0 + kCT < Cin) load_slice(c0 + kCT);
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap % 3;
      bf16x8 B[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t)
        B[t] = *reinterpret_cast<const bf16x8*>(swt + (tap * 16 * NT + t * 16 + (lane & 15)) * kCTP + kq);
#pragma unroll
      for (int q = 0; q < RW; ++q) {
        const int rloc = wv * RW + q;   // output row within the block
        if (h0 + rloc >= H) continue;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const bf16x8 A =
              *reinterpret_cast<const bf16x8*>(sx + ((rloc + dy) * 66 + g * 16 + (lane & 15) + dx) * kCTP + kq);
#pragma unroll
          for (int t = 0; t < NT; ++t) acc[q][g][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B[t], acc[q][g][t], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RW; ++q) {
    const int h = h0 + wv * RW + q;
    if (h >= H) continue;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int co = co_base + t * 16 + (lane & 15);
      if (co >= Cout) continue;
      const float b = bv[t];
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int px = pbase + g * 16 + (lane >> 4) * 4 + r;
          if (px >= W) continue;
          float v = acc[q][g][t][r] + b;
          if (relu) v = fmaxf(v, 0.f);
          store1(y + ((int64_t)h * W + px) * Cout + co, v);
        }
    }
  }
  if (RW == 1 && ypool) {
    // 2 x 2 average pooling of the stored (rounded) output into ypool (H/2 x W/2), in
    // the order of the separate pooling kernel: s = 0; s += y(2i, 2j), y(2i, 2j+1),
    // y(2i+1, 2j), y(2i+1, 2j+1); out = round(s / 4).  Wave w holds row h0 + w: the odd
    // wave of each pair passes its rounded values to the even one through the input
    // tile's LDS, which the last slice's MFMAs no longer read.
    uint16_t* xch = sx;   // [2 pairs][4 pixel groups][NT][4][64 lanes]
    const int pair = wv >> 1;
    __syncthreads();
    if (wv & 1) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int co = co_base + t * 16 + (lane & 15);
        const float b = bv[t];
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float v = acc[0][g][t][r] + b;
            if (relu) v = fmaxf(v, 0.f);
            xch[(((pair * 4 + g) * NT + t) * 4 + r) * 64 + lane] = co < Cout ? f2bf(v) : (uint16_t)0;
          }
      }
    }
    __syncthreads();
    const int h = h0 + wv;
    if (!(wv & 1) && h + 1 < H) {
      const int Wo = W >> 1;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int co = co_base + t * 16 + (lane & 15);
        if (co >= Cout) continue;
        const float b = bv[t];
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
          for (int r = 0; r < 4; r += 2) {
            const int px = pbase + g * 16 + (lane >> 4) * 4 + r;
            if (px + 1 >= W) continue;
            float v0 = acc[0][g][t][r] + b, v1 = acc[0][g][t][r + 1] + b;
            if (relu) {
              v0 = fmaxf(v0, 0.f);
              v1 = fmaxf(v1, 0.f);
            }
            const int base = (((pair * 4 + g) * NT + t) * 4 + r) * 64 + lane;
            float sum = 0.f;
            sum += bf2f(f2bf(v0));
            sum += bf2f(f2bf(v1));
            sum += bf2f(xch[base]);
            sum += bf2f(xch[base + 64]);
            store1(ypool + ((int64_t)(h >> 1) * Wo + (px >> 1)) * Cout + co, 0.25f * sum);
          }
      }
    }
  }
}

// output-channel tiles per block for Cout channels: 16 NT channels, NT <= 4
// output-channel tile (16 nt channels) of a convolution: the widest that covers Cout,
// narrowed while the launch has fewer than 256 blocks (the lower levels of the network
// would otherwise leave most CUs idle: 16 blocks for 64 x 64 channels at 64^2)
static inline int conv_nt(int H, int W, int cout) {
  int nt = cout >= 64 ? 4 : (cout + 15) / 16;
  const int64_t px_blocks =
      (int64_t)((W + 63) / 64) * ((H + 4 * kConvRowsPerWave - 1) / (4 * kConvRowsPerWave));
  while (nt > 1 && px_blocks * ((cout + 16 * nt - 1) / (16 * nt)) < 256) nt = nt == 4 ? 2 : 1;
  return nt;
}

template <typename TIN, typename TOUT>
static void launch_conv3t(int H, int W, const TIN* x0, int C0, int up0, const TIN* x1, int C1, const uint16_t* w,
                          const float* bias, int Cout, TOUT* y, int relu, const int* skip, hipStream_t s,
                          TOUT* ypool = nullptr) {
  const int nt = conv_nt(H, W, Cout);
  constexpr int RW = kConvRowsPerWave;
  dim3 grd((W + 63) / 64, (H + 4 * RW - 1) / (4 * RW), (Cout + 16 * nt - 1) / (16 * nt));
  switch (nt) {
    case 1: k_conv3t<1, RW, TIN, TOUT><<<grd, 256, 0, s>>>(H, W, x0, C0, up0, x1, C1, w, bias, Cout, y, relu, skip, ypool); break;
    case 2: k_conv3t<2, RW, TIN, TOUT><<<grd, 256, 0, s>>>(H, W, x0, C0, up0, x1, C1, w, bias, Cout, y, relu, skip, ypool); break;
    case 3: k_conv3t<3, RW, TIN, TOUT><<<grd, 256, 0, s>>>(H, W, x0, C0, up0, x1, C1, w, bias, Cout, y, relu, skip, ypool); break;
    default: k_conv3t<4, RW, TIN, TOUT><<<grd, 256, 0, s>>>(H, W, x0, C0, up0, x1, C1, w, bias, Cout, y, relu, skip, ypool); break;
  }
}

// ---------------------------------------------------------------------------
// weight gradient: part[chunk][tap][co][ci] = sum_{p in chunk} gT[co][p] * xs_tap[p][ci]
// xT: channel-major input (Cin x HW), gT: channel-major output gradient (Cout x HW).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_wgrad3(int H, int W, const uint16_t* __restrict__ xT, int Cin,
                                                const uint16_t* __restrict__ gT, int Cout, int chunk,
                                                float* __restrict__ part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tap = blockIdx.y;
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  const int nco = (Cout + 63) / 64;
  const int co_blk = blockIdx.x % nco, ci_blk = blockIdx.x / nco;
  const int HW = H * W;
  const int p0 = blockIdx.z * chunk;
  const int p1 = min(p0 + chunk, HW);
  const int co_row = co_blk * 64 + wv * 16 + (lane & 15);
  const int kq = (lane >> 4) * 4;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int pk = p0; pk < p1; pk += 16) {
    bf16x4 A = {0, 0, 0, 0};
    int hs[4], ws[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = pk + kq + r;
      hs[r] = -1;
      if (p < p1) {
        if (co_row < Cout) A[r] = (short)gT[(int64_t)co_row * HW + p];
        const int hh = p / W + dy, ww = p % W + dx;
        if (hh >= 0 && hh < H && ww >= 0 && ww < W) {
          hs[r] = hh;
          ws[r] = ww;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int ci = ci_blk * 64 + t * 16 + (lane & 15);
      bf16x4 B = {0, 0, 0, 0};
      if (ci < Cin) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (hs[r] >= 0) B[r] = (short)xT[(int64_t)ci * HW + hs[r] * W + ws[r]];
      }
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int ci = ci_blk * 64 + t * 16 + (lane & 15);
    if (ci >= Cin) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int co = co_blk * 64 + wv * 16 + (lane >> 4) * 4 + r;
      if (co < Cout) part[(((int64_t)blockIdx.z * 9 + tap) * Cout + co) * Cin + ci] = acc[t][r];
    }
  }
}

// ---------------------------------------------------------------------------
// Weight and bias gradient on the K = 32 MFMA: part[chunk][tap][co][ci] =
// sum_{p in chunk} gT[co][p] * x(p shifted by the tap)[ci], bpart[chunk][co] =
// sum_{p in chunk} gT[co][p].  M = output channels, N = input channels, K = pixels:
// each lane supplies 8 consecutive pixels of one output channel (A) and of one input
// channel (B), as 16-byte loads.  The input comes as three copies shifted by dx =
// -1, 0, +1 within each row (zero beyond the row's ends), so that every tap's B is an
// aligned 8-pixel run of one copy at an offset of dy rows.  A block owns 64 output x 16
// input channels and one pixel chunk; each of its four waves takes every fourth
// 32-pixel step of the chunk for all nine taps (36 accumulator tiles, so one A load
// serves nine taps and one B load four output tiles), loading the next step while the
// current one multiplies, and the waves are summed through LDS in a fixed order.
// Requires W % 8 == 0 and chunk % 128 == 0.
// ---------------------------------------------------------------------------
constexpr int kWgradBlocks = 512;   // workgroups a weight-gradient launch aims for

__global__ __launch_bounds__(256) void k_wgrad3t(int H, int W, const uint16_t* __restrict__ xTs, int Cin,
                                                 const uint16_t* __restrict__ gT, int Cout, int chunk,
                                                 float* __restrict__ part, float* __restrict__ bpart) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nco = (Cout + 63) / 64;
  const int co_blk = blockIdx.x % nco, ci_blk = blockIdx.x / nco;
  const int64_t HW = (int64_t)H * W;
  const int64_t p0 = (int64_t)blockIdx.z * chunk;
  const int64_t p1 = min(p0 + (int64_t)chunk, HW);
  const int kq = (lane >> 4) * 8;
  const int ci = ci_blk * 16 + (lane & 15);
  const bool ci_ok = ci < Cin;
  const bool do_bias = ci_blk == 0;
  const uint16_t* arow[4];
  bool co_ok[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int co = co_blk * 64 + t * 16 + (lane & 15);
    co_ok[t] = co < Cout;
    arow[t] = gT + (int64_t)(co_ok[t] ? co : 0) * HW;
  }
  const uint16_t* brow[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) brow[s] = xTs + ((int64_t)s * Cin + (ci_ok ? ci : 0)) * HW;
  const bf16x8 zero = __builtin_bit_cast(bf16x8, make_uint4(0u, 0u, 0u, 0u));
  // one 32-pixel step: this lane's 8 pixels (within one row, as W % 8 == 0), masked
  // outside the chunk, the channel range and the image rows
  auto load_step = [&](int64_t pk, bf16x8(&A)[4], bf16x8(&B)[9]) {
    const int64_t p = pk + kq;
    const bool p_ok = p < p1;
    const int h = (int)(p / W);
#pragma unroll
    for (int t = 0; t < 4; ++t) A[t] = (p_ok && co_ok[t]) ? load8(arow[t] + p) : zero;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const bool row_ok = p_ok && ci_ok && h + dy >= 0 && h + dy < H;
#pragma unroll
      for (int s = 0; s < 3; ++s) B[(dy + 1) * 3 + s] = row_ok ? load8(brow[s] + p + (int64_t)dy * W) : zero;
    }
  };
  f32x4 acc[9][4];
#pragma unroll
  for (int tp = 0; tp < 9; ++tp)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[tp][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum[4] = {0.f, 0.f, 0.f, 0.f};
  bf16x8 A[4], B[9];
  int64_t pk = p0 + wv * 32;
  load_step(pk, A, B);
  for (; pk < p1; pk += 128) {
    bf16x8 An[4], Bn[9];
    load_step(pk + 128, An, Bn);
    if (do_bias) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int e = 0; e < 8; ++e) bsum[t] += (float)A[t][e];
    }
#pragma unroll
    for (int tp = 0; tp < 9; ++tp)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[tp][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[t], B[tp], acc[tp][t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < 4; ++t) A[t] = An[t];
#pragma unroll
    for (int b = 0; b < 9; ++b) B[b] = Bn[b];
  }
  // sum the four waves, one tap at a time: accumulator r of tile t in lane l is
  // output channel t*16 + (l/16)*4 + r and input channel l % 16
  __shared__ float red[4][64][17];
  for (int tp = 0; tp < 9; ++tp) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wv][lane][t * 4 + r] = acc[tp][t][r];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = threadIdx.x + 256 * j;
      const int ci_l = e & 15, co_l = e >> 4;
      const int src = ((co_l >> 2) & 3) * 16 + ci_l, slot = (co_l >> 4) * 4 + (co_l & 3);
      const float v = red[0][src][slot] + red[1][src][slot] + red[2][src][slot] + red[3][src][slot];
      const int co = co_blk * 64 + co_l, cig = ci_blk * 16 + ci_l;
      if (co < Cout && cig < Cin) part[(((int64_t)blockIdx.z * 9 + tp) * Cout + co) * Cin + cig] = v;
    }
    __syncthreads();
  }
  if (do_bias) {
    // lanes l, l ^ 16, l ^ 32, l ^ 48 hold the same output channel's sums over their pixels
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      float v = bsum[t];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (lane < 16) red[wv][t * 16 + lane][0] = v;
    }
    __syncthreads();
    const int co = co_blk * 64 + (int)threadIdx.x;
    if (threadIdx.x < 64 && co < Cout)
      bpart[(int64_t)blockIdx.z * Cout + co] =
          red[0][threadIdx.x][0] + red[1][threadIdx.x][0] + red[2][threadIdx.x][0] + red[3][threadIdx.x][0];
  }
}

// Channel-major copies for the weight gradients, through a 64-pixel x 32-channel LDS
// tile so that reads (pixel-major rows of channels) and writes (channel-major runs of
// pixels) are both 16-byte and coalesced.  Pixels p0 .. p0 + 63 of the flattened image
// plus one pixel either side; grid (ceil(HW / 64), ceil(C / 32)).  Requires W % 8 == 0
// and channel counts that are multiples of 8.
constexpr int kTrPix = 64, kTrCh = 32, kTrPad = kTrCh + 2;

__device__ __forceinline__ uint4 pack8(const uint16_t (&v)[8]) {
  return make_uint4(v[0] | ((uint32_t)v[1] << 16), v[2] | ((uint32_t)v[3] << 16), v[4] | ((uint32_t)v[5] << 16),
                    v[6] | ((uint32_t)v[7] << 16));
}

// the input of a conv3 layer (x0, optionally 2x-upsampled, concatenated with x1) as three
// channel-major copies shifted by dx = -1, 0, +1 within each row:
// out[s][c][p] = x(h, w + s - 1)[c], zero beyond the row's ends
__global__ __launch_bounds__(256) void k_to_chw3(int H, int W, const uint16_t* __restrict__ x0, int C0, int up0,
                                                 const uint16_t* __restrict__ x1, int C1, uint16_t* __restrict__ out) {
  __shared__ uint16_t tile[kTrPix + 2][kTrPad];
  const int HW = H * W, C = C0 + C1, W0 = up0 ? W / 2 : W;
  const int p0 = blockIdx.x * kTrPix, c0 = blockIdx.y * kTrCh;
  for (int i = threadIdx.x; i < (kTrPix + 2) * (kTrCh / 8); i += 256) {
    const int q = p0 - 1 + i / (kTrCh / 8), k = c0 + (i % (kTrCh / 8)) * 8;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (q >= 0 && q < HW && k < C) {
      const int h = q / W, w = q % W;
      if (k < C0) v = *reinterpret_cast<const uint4*>(x0 + (up0 ? (int64_t)(h / 2) * W0 + w / 2 : (int64_t)q) * C0 + k);
      else v = *reinterpret_cast<const uint4*>(x1 + (int64_t)q * C1 + (k - C0));
    }
    uint16_t* t = &tile[i / (kTrCh / 8)][(i % (kTrCh / 8)) * 8];
    t[0] = v.x & 0xffff; t[1] = v.x >> 16; t[2] = v.y & 0xffff; t[3] = v.y >> 16;
    t[4] = v.z & 0xffff; t[5] = v.z >> 16; t[6] = v.w & 0xffff; t[7] = v.w >> 16;
  }
  __syncthreads();
  // 3 copies x 32 channels x 8 groups of 8 pixels
  for (int i = threadIdx.x; i < 3 * kTrCh * (kTrPix / 8); i += 256) {
    const int g = i % (kTrPix / 8), c = (i / (kTrPix / 8)) % kTrCh, s = i / (kTrCh * (kTrPix / 8));
    const int p = p0 + g * 8;
    if (p >= HW || c0 + c >= C) continue;
    const int w = p % W;   // the 8 pixels share a row (W % 8 == 0)
    uint16_t v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int ws = w + e + s - 1;
      v[e] = (ws >= 0 && ws < W) ? tile[g * 8 + e + s][c] : (uint16_t)0;
    }
    *reinterpret_cast<uint4*>(out + ((int64_t)s * C + c0 + c) * HW + p) = pack8(v);
  }
}

// ReLU backward with the channel-major BF16 copy for the weight gradient:
// gpre = g where the layer's output is positive, else 0 (pixel-major, FP32), and
// gT[c][p] = bf16(gpre[p][c]).  Same tiling as k_to_chw3 (no halo); requires HW % 8 == 0
// and C % 8 == 0.
__global__ __launch_bounds__(256) void k_relu_grad_t(int HW, int C, const float* __restrict__ g,
                                                     const uint16_t* __restrict__ outv, float* __restrict__ gpre,
                                                     uint16_t* __restrict__ gT) {
  __shared__ uint16_t tile[kTrPix][kTrPad];
  const int p0 = blockIdx.x * kTrPix, c0 = blockIdx.y * kTrCh;
  // 64 pixels x 32 channels, 4 channels per thread and pass
  for (int i = threadIdx.x; i < kTrPix * (kTrCh / 4); i += 256) {
    const int pl = i / (kTrCh / 4), k = (i % (kTrCh / 4)) * 4;
    const int p = p0 + pl, c = c0 + k;
    if (p >= HW || c >= C) continue;
    const int64_t o = (int64_t)p * C + c;
    const float4 gv = *reinterpret_cast<const float4*>(g + o);
    const uint2 ov = *reinterpret_cast<const uint2*>(outv + o);
    float4 r;
    r.x = bf2f(ov.x & 0xffff) > 0.f ? gv.x : 0.f;
    r.y = bf2f(ov.x >> 16) > 0.f ? gv.y : 0.f;
    r.z = bf2f(ov.y & 0xffff) > 0.f ? gv.z : 0.f;
    r.w = bf2f(ov.y >> 16) > 0.f ? gv.w : 0.f;
    *reinterpret_cast<float4*>(gpre + o) = r;
    tile[pl][k] = f2bf(r.x); tile[pl][k + 1] = f2bf(r.y); tile[pl][k + 2] = f2bf(r.z); tile[pl][k + 3] = f2bf(r.w);
  }
  __syncthreads();
  // 32 channels x 8 groups of 8 pixels
  {
    const int i = threadIdx.x;
    const int gp = i % (kTrPix / 8), c = i / (kTrPix / 8);
    const int p = p0 + gp * 8;
    if (p < HW && c0 + c < C) {
      uint16_t v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = tile[gp * 8 + e][c];
      *reinterpret_cast<uint4*>(gT + (int64_t)(c0 + c) * HW + p) = pack8(v);
    }
  }
}

// sum over chunks in a fixed order: out[i] = sum_c part[c * n + i].  A block covers 32
// consecutive i; its 8 thread rows take every eighth chunk and meet in LDS.
__global__ __launch_bounds__(256) void k_sum_chunks(const float* __restrict__ part, int nchunks, int64_t n,
                                                    float* __restrict__ out) {
  const int tx = threadIdx.x & 31, gr = threadIdx.x >> 5;
  const int64_t i = (int64_t)blockIdx.x * 32 + tx;
  float s = 0.f;
  if (i < n) {
#pragma unroll 4
    for (int c = gr; c < nchunks; c += 8) s += part[(int64_t)c * n + i];
  }
  __shared__ float red[8][33];
  red[gr][tx] = s;
  __syncthreads();
  if (gr == 0 && i < n) {
    float t = red[0][tx];
#pragma unroll
    for (int k = 1; k < 8; ++k) t += red[k][tx];
    out[i] = t;
  }
}

// row sums of a channel-major tensor: out[c] = sum_p g[c][p]  (bias gradient)
__global__ void k_rowsum(const uint16_t* __restrict__ gT, int HW, float* __restrict__ out) {
  const int c = blockIdx.x;
  float s = 0.f;
  for (int p = threadIdx.x; p < HW; p += blockDim.x) s += bf2f(gT[(int64_t)c * HW + p]);
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

// ---------------------------------------------------------------------------
// elementwise / layout helpers
// ---------------------------------------------------------------------------
// pack an (HW x cin) FP32 tensor into (HW x cpad) bf16 with zero channels
__global__ void k_pack(int64_t npix, const float* __restrict__ x, int cin, int cpad, uint16_t* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npix * cpad; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = i / cpad;
    const int c = (int)(i % cpad);
    out[i] = c < cin ? f2bf(x[p * cin + c]) : (uint16_t)0;
  }
}

__global__ void k_pool2(int Ho, int Wo, int C, const uint16_t* __restrict__ in, uint16_t* __restrict__ out,
                        const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t n = (int64_t)Ho * Wo * C;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    const int64_t p = i / C;
    const int wo = (int)(p % Wo), ho = (int)(p / Wo);
    const int Wi = 2 * Wo;
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) s += bf2f(in[((int64_t)(2 * ho + a) * Wi + 2 * wo + b) * C + c]);
    out[i] = f2bf(0.25f * s);
  }
}

// channel-major bf16 copy of the (optionally concatenated / upsampled) conv input
__global__ void k_to_chw(int H, int W, const uint16_t* __restrict__ x0, int C0, int up0,
                         const uint16_t* __restrict__ x1, int C1, uint16_t* __restrict__ out) {
  const int64_t HW = (int64_t)H * W;
  const int C = C0 + C1;
  const int W0 = up0 ? W / 2 : W;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < HW * C; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i / HW);
    const int64_t p = i % HW;
    const int h = (int)(p / W), w = (int)(p % W);
    uint16_t v;
    if (c < C0) v = up0 ? x0[((int64_t)(h / 2) * W0 + w / 2) * C0 + c] : x0[p * C0 + c];
    else v = x1[p * C1 + (c - C0)];
    out[i] = v;
  }
}

// gradient through ReLU: gpre = g * (out > 0); NHWC FP32 copy and channel-major bf16 copy
__global__ void k_relu_grad(int64_t HW, int C, const float* __restrict__ g, const uint16_t* __restrict__ outv,
                            float* __restrict__ gpre, uint16_t* __restrict__ gT) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < HW * C; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = i / C;
    const int c = (int)(i % C);
    const float v = bf2f(outv[i]) > 0.f ? g[i] : 0.f;
    gpre[i] = v;
    gT[(int64_t)c * HW + p] = f2bf(v);
  }
}

// split the gradient of concat(up2(d), skip): gd[hh][ww][c] = sum of the 2x2 block
// (c < Cu); gskip[h][w][c] = gcat[h][w][Cu + c]
__global__ void k_split_cat(int H, int W, int Cu, int Cs, const float* __restrict__ gcat, float* __restrict__ gd,
                            float* __restrict__ gskip) {
  const int C = Cu + Cs;
  const int64_t nhalf = (int64_t)(H / 2) * (W / 2) * Cu;
  const int64_t nfull = (int64_t)H * W * Cs;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nhalf + nfull; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < nhalf) {
      const int c = (int)(i % Cu);
      const int64_t q = i / Cu;
      const int wo = (int)(q % (W / 2)), ho = (int)(q / (W / 2));
      float s = 0.f;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) s += gcat[((int64_t)(2 * ho + a) * W + 2 * wo + b) * C + c];
      gd[i] = s;
    } else {
      const int64_t j = i - nhalf;
      const int c = (int)(j % Cs);
      const int64_t p = j / Cs;
      gskip[j] = gcat[p * C + Cu + c];
    }
  }
}

// ge[h][w][c] += 0.25 * ga[h/2][w/2][c]  (average-pool backward), optionally ge = gadd + ...
__global__ void k_pool_back_add(int H, int W, int C, const float* __restrict__ ga, const float* __restrict__ gadd,
                                float* __restrict__ ge) {
  const int64_t n = (int64_t)H * W * C;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    const int64_t p = i / C;
    const int w = (int)(p % W), h = (int)(p / W);
    ge[i] = gadd[i] + 0.25f * ga[((int64_t)(h / 2) * (W / 2) + w / 2) * C + c];
  }
}

// 1x1 head (FP32): y[p][co] = b[co] + sum_ci x[p][ci] * w[co][ci]
// 1x1 head: y[p][co] = b[co] + sum_ci x[p][ci] w[co][ci], summed in channel order.  One
// pixel per thread, its channels as 16-byte loads; MAXCO bounds Cout.  Requires Cin % 8 == 0.
template <int MAXCO>
__global__ __launch_bounds__(256) void k_head_fwd(int64_t npix, const uint16_t* __restrict__ x, int Cin,
                                                  const float* __restrict__ w, const float* __restrict__ b, int Cout,
                                                  float* __restrict__ y, const int* __restrict__ skip) {
  if (skip && *skip) return;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x) {
    float s[MAXCO];
#pragma unroll
    for (int co = 0; co < MAXCO; ++co) s[co] = co < Cout ? b[co] : 0.f;
    for (int c8 = 0; c8 < Cin; c8 += 8) {
      const bf16x8 xv = load8(x + p * Cin + c8);
#pragma unroll
      for (int co = 0; co < MAXCO; ++co) {
        if (co < Cout) {
#pragma unroll
          for (int e = 0; e < 8; ++e) s[co] += (float)xv[e] * w[co * Cin + c8 + e];
        }
      }
    }
#pragma unroll
    for (int co = 0; co < MAXCO; ++co)
      if (co < Cout) y[p * Cout + co] = s[co];
  }
}

__global__ void k_head_dx(int64_t npix, const float* __restrict__ gy, int Cout, const float* __restrict__ w, int Cin,
                          float* __restrict__ gx) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npix * Cin; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = i / Cin;
    const int ci = (int)(i % Cin);
    float s = 0.f;
    for (int co = 0; co < Cout; ++co) s += gy[p * Cout + co] * w[co * Cin + ci];
    gx[i] = s;
  }
}

// head weight/bias gradient: one block per (co, ci) pair (ci = Cin means the bias)
// Head (1x1) weight and bias gradient partials over a pixel range of ppb pixels:
// part[blk][co * Cin + ci] = sum_p gy[p][co] x[p][ci] and part[blk][Cout * Cin + co] =
// sum_p gy[p][co].  blockIdx.y picks an 8-channel slice of x (one 16-byte load per
// pixel, consecutive threads on consecutive pixels); the bias sums ride on slice 0.
// MAXCO bounds Cout.  Requires Cin % 8 == 0.
template <int MAXCO>
__global__ __launch_bounds__(256) void k_head_dw_part(int64_t npix, int ppb, const float* __restrict__ gy, int Cout,
                                                      const uint16_t* __restrict__ x, int Cin,
                                                      float* __restrict__ part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c0 = blockIdx.y * 8;
  const int64_t p0 = (int64_t)blockIdx.x * ppb;
  const int64_t p1 = min(p0 + (int64_t)ppb, npix);
  float acc[MAXCO][9];
#pragma unroll
  for (int co = 0; co < MAXCO; ++co)
#pragma unroll
    for (int e = 0; e < 9; ++e) acc[co][e] = 0.f;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) {
    const bf16x8 xv = load8(x + p * Cin + c0);
#pragma unroll
    for (int co = 0; co < MAXCO; ++co) {
      const float g = co < Cout ? gy[p * Cout + co] : 0.f;
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[co][e] += g * (float)xv[e];
      acc[co][8] += g;
    }
  }
  __shared__ float red[4][MAXCO * 9];
#pragma unroll
  for (int co = 0; co < MAXCO; ++co)
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      float v = acc[co][e];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) red[wv][co * 9 + e] = v;
    }
  __syncthreads();
  const int i = threadIdx.x;
  if (i < MAXCO * 9) {
    const int co = i / 9, e = i % 9;
    if (co < Cout && (e < 8 || blockIdx.y == 0)) {
      const float v = red[0][i] + red[1][i] + red[2][i] + red[3][i];
      const int64_t base = (int64_t)blockIdx.x * (Cout * Cin + Cout);
      part[base + (e < 8 ? (int64_t)co * Cin + c0 + e : (int64_t)Cout * Cin + co)] = v;
    }
  }
}

// relative loss: sums of (y - t)^2 and t^2 per block, then the gradient 2 (y - t) / sum t^2
__global__ void k_loss_part(int64_t n, const float* __restrict__ y, const float* __restrict__ t,
                            double* __restrict__ part) {
  double a = 0.0, b = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double d = (double)y[i] - (double)t[i];
    a += d * d;
    b += (double)t[i] * (double)t[i];
  }
  __shared__ double ra[256], rb[256];
  ra[threadIdx.x] = a;
  rb[threadIdx.x] = b;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      ra[threadIdx.x] += ra[threadIdx.x + o];
      rb[threadIdx.x] += rb[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ra[0];
    part[2 * blockIdx.x + 1] = rb[0];
  }
}

__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  __shared__ double ra[256], rb[256];
  ra[threadIdx.x] = a;
  rb[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      ra[threadIdx.x] += ra[threadIdx.x + o];
      rb[threadIdx.x] += rb[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = rb[0] > 0 ? ra[0] / rb[0] : 0.0;
    out[1] = rb[0];
  }
}

__global__ void k_loss_grad(int64_t n, const float* __restrict__ y, const float* __restrict__ t,
                            const double* __restrict__ sums, float* __restrict__ gy) {
  const float sc = sums[1] > 0 ? (float)(2.0 / sums[1]) : 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    gy[i] = sc * (y[i] - t[i]);
}

__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// bf16 forward weights (same layout as the master) and input-gradient weights
// wt[tap][ci][co] = w[8 - tap][co][ci]
__global__ void k_weights_bf16(int Cout, int Cin, const float* __restrict__ wm, uint16_t* __restrict__ wf,
                               uint16_t* __restrict__ wt) {
  const int64_t n = (int64_t)9 * Cout * Cin;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int ci = (int)(i % Cin);
    const int co = (int)((i / Cin) % Cout);
    const int tap = (int)(i / ((int64_t)Cin * Cout));
    const uint16_t v = f2bf(wm[i]);
    wf[i] = v;
    wt[((int64_t)(8 - tap) * Cin + ci) * Cout + co] = v;
  }
}

static int64_t grid_for(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }
// k_sum_chunks: one block per 32 outputs
static unsigned sum_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 31) / 32); }

}  // namespace m1

using namespace m1;

// ============================================================================
// Host-side network object
// ============================================================================
namespace {

struct ConvLayer {
  int cin, cout;        // cin padded to a multiple of 16 (conv3)
  int cin_true;         // channels of the unpadded definition
  int64_t woff, boff;   // offsets in the parameter slab (FP32)
  int64_t wsize;
  uint16_t* wf = nullptr;   // bf16 forward weights
  uint16_t* wt = nullptr;   // bf16 input-gradient weights
};

}  // namespace

struct m1nn {
  int cin = 0, cin_pad = 0, cout = 0, L = 0;
  int ch[8] = {};
  int Hmax = 0, Wmax = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<ConvLayer> conv;   // enc0a, enc0b, ..., dec(L-2)a, dec(L-2)b, ..., dec0a, dec0b
  int64_t nparam = 0;            // FP32 slab length (padded layout)
  float* P = nullptr;            // master parameters
  float* G = nullptr;            // gradients
  float* Mo = nullptr;           // Adam first moment
  float* Vo = nullptr;           // Adam second moment
  int adam_t = 0;
  int64_t head_w = 0, head_b = 0;
  // activations (bf16 NHWC) per level
  uint16_t* in = nullptr;
  std::vector<uint16_t*> ha, e, a, hd, d;   // ha_l, e_l, a_{l} (pooled input of level l, l>=1), hd_l, d_l
  float* y = nullptr;
  // backward buffers
  float* gy = nullptr;
  float* gbuf0 = nullptr;   // FP32 scratch sized for the largest tensor
  float* gbuf1 = nullptr;
  float* gbuf2 = nullptr;
  float* gpre = nullptr;
  std::vector<float*> genc; // gradient w.r.t. e_l (FP32)
  uint16_t* xT = nullptr;   // channel-major input copy for wgrad
  uint16_t* gT = nullptr;   // channel-major gradient copy for wgrad
  float* wpart = nullptr;
  int64_t wpart_len = 0;
  float* bpart = nullptr;   // per-chunk bias-gradient partials
  double* loss_part = nullptr;
  double* loss_out = nullptr;
  const int* skip = nullptr;  // device flag: forward kernels return at once when it is set
};

namespace {

int conv_index(const m1nn* n, const char kind, int level, int ab) {
  // kind 'e' encoder, 'd' decoder; ab 0 = first conv, 1 = second
  if (kind == 'e') return 2 * level + ab;
  // decoder levels are stored L-2 down to 0
  return 2 * n->L + 2 * (n->L - 2 - level) + ab;
}

bool ok(m1nn* n, hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  n->err = std::string(what) + ": " + hipGetErrorString(e);
  return false;
}

template <typename T> bool alloc(m1nn* n, T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) return true;
  return ok(n, hipMalloc((void**)p, sizeof(T) * (size_t)count), "hipMalloc");
}

void nn_free(m1nn* n) {
  auto f = [](void* p) { if (p) hipFree(p); };
  for (auto& c : n->conv) { f(c.wf); f(c.wt); }
  f(n->P); f(n->G); f(n->Mo); f(n->Vo); f(n->in); f(n->y); f(n->gy); f(n->gbuf0); f(n->gbuf1); f(n->gbuf2);
  f(n->gpre); f(n->xT); f(n->gT); f(n->wpart); f(n->bpart); f(n->loss_part); f(n->loss_out);
  for (auto* p : n->ha) f(p);
  for (auto* p : n->e) f(p);
  for (auto* p : n->a) f(p);
  for (auto* p : n->hd) f(p);
  for (auto* p : n->d) f(p);
  for (auto* p : n->genc) f(p);
}

void refresh_weights(m1nn* n) {
  for (auto& c : n->conv) {
    const int64_t cnt = (int64_t)9 * c.cout * c.cin;
    k_weights_bf16<<<grid_for(cnt), 256, 0, n->stream>>>(c.cout, c.cin, n->P + c.woff, c.wf, c.wt);
  }
}

// K = 32 kernel (weights staged in LDS) when the channels fit; the K = 16 kernel otherwise
static bool use_k32(int cin) {
  static int v = -1;
  if (v < 0) {
    const char* e = getenv("M1_CONV_KERNEL");
    v = (e && std::string(e) == "k16") ? 0 : 1;
  }
  return v == 1 && cin % 16 == 0;
}

// y = relu(conv3(x)); with ypool (H and W even), also its 2 x 2 average pooling.
// Returns whether ypool was written (the K = 16 kernel leaves it to the caller).
bool conv3(m1nn* n, int H, int W, const uint16_t* x0, int C0, int up0, const uint16_t* x1, int C1, const ConvLayer& c,
           uint16_t* y, int relu, uint16_t* ypool = nullptr) {
  if (use_k32(C0 + C1) && C0 % 8 == 0) {
    launch_conv3t<uint16_t, uint16_t>(H, W, x0, C0, up0, x1, C1, c.wf, n->P + c.boff, c.cout, y, relu, n->skip,
                                      n->stream, ypool);
    return ypool != nullptr;
  }
  dim3 grd((W + 63) / 64, H, (c.cout + 63) / 64);
  k_conv3<uint16_t, uint16_t><<<grd, 256, 0, n->stream>>>(H, W, x0, C0, up0, x1, C1, c.wf, n->P + c.boff, c.cout, y,
                                                          relu, n->skip);
  return false;
}

// input gradient of a conv3 layer: gx (H, W, cin) FP32 from gpre (H, W, cout) FP32
void conv3_dgrad(m1nn* n, int H, int W, const float* gpre, const ConvLayer& c, float* gx) {
  if (use_k32(c.cout)) {
    launch_conv3t<float, float>(H, W, gpre, c.cout, 0, nullptr, 0, c.wt, nullptr, c.cin, gx, 0, nullptr, n->stream);
    return;
  }
  dim3 grd((W + 63) / 64, H, (c.cin + 63) / 64);
  k_conv3<float, float><<<grd, 256, 0, n->stream>>>(H, W, gpre, c.cout, 0, nullptr, 0, c.wt, nullptr, c.cin, gx, 0,
                                                    nullptr);
}

// the K = 32 weight gradient applies when image rows are whole 8-pixel groups
static bool wgrad_k32(int W) { return W % 8 == 0; }

// pixel chunk of the K = 32 weight gradient: a multiple of 128 pixels (a 32-pixel step
// for each of a block's four waves) such that blocks x chunks is about kWgradBlocks;
// the number of chunks is at most max(1, kWgradBlocks / blocks)
static int wgrad_chunk(int64_t HW, int blocks, int* nch) {
  const int64_t target = std::max<int64_t>(1, kWgradBlocks / blocks);
  int64_t chunk = (HW + target - 1) / target;
  chunk = std::max<int64_t>(128, (chunk + 127) / 128 * 128);
  *nch = (int)((HW + chunk - 1) / chunk);
  return (int)chunk;
}

// pixels per block of the head weight gradient: at most 256 blocks
static int head_ppb(int64_t npix) { return (int)std::max<int64_t>(256, ((npix + 255) / 256 + 255) / 256 * 256); }

// weight and bias gradient of a conv3 layer from xT (cin x HW, or its three dx-shifted
// copies for the K = 32 kernel) and gT (cout x HW)
void conv3_wgrad(m1nn* n, int H, int W, const ConvLayer& c) {
  const int64_t HW = (int64_t)H * W;
  const int64_t nw = (int64_t)9 * c.cout * c.cin;
  if (wgrad_k32(W)) {
    const int blocks = ((c.cout + 63) / 64) * ((c.cin + 15) / 16);
    int nch = 0;
    const int chunk = wgrad_chunk(HW, blocks, &nch);
    k_wgrad3t<<<dim3(blocks, 1, nch), 256, 0, n->stream>>>(H, W, n->xT, c.cin, n->gT, c.cout, chunk, n->wpart,
                                                            n->bpart);
    k_sum_chunks<<<sum_grid(nw), 256, 0, n->stream>>>(n->wpart, nch, nw, n->G + c.woff);
    k_sum_chunks<<<sum_grid(c.cout), 256, 0, n->stream>>>(n->bpart, nch, c.cout, n->G + c.boff);
    return;
  }
  const int chunk = 4096;
  const int nch = (int)((HW + chunk - 1) / chunk);
  const int blocks = ((c.cout + 63) / 64) * ((c.cin + 63) / 64);
  k_wgrad3<<<dim3(blocks, 9, nch), 256, 0, n->stream>>>(H, W, n->xT, c.cin, n->gT, c.cout, chunk, n->wpart);
  k_sum_chunks<<<sum_grid(nw), 256, 0, n->stream>>>(n->wpart, nch, nw, n->G + c.woff);
  k_rowsum<<<c.cout, 256, 0, n->stream>>>(n->gT, HW, n->G + c.boff);
}

// the features the 1x1 head reads: the top decoder output, or with a single level
// (no decoder) the top encoder output, as d_{L-1} = e_{L-1} at the bottom
static const uint16_t* head_input(const m1nn* n) { return n->L > 1 ? n->d[0] : n->e[0]; }

void forward_impl(m1nn* n, int H, int W) {
  const int L = n->L;
  const uint16_t* a = n->in;
  int cprev = n->cin_pad;
  for (int l = 0; l < L; ++l) {
    const int Hl = H >> l, Wl = W >> l;
    const ConvLayer& ca = n->conv[conv_index(n, 'e', l, 0)];
    const ConvLayer& cb = n->conv[conv_index(n, 'e', l, 1)];
    conv3(n, Hl, Wl, a, cprev, 0, nullptr, 0, ca, n->ha[l], 1);
    // the level's output, pooled in the same launch for the next level
    const bool pooled = conv3(n, Hl, Wl, n->ha[l], n->ch[l], 0, nullptr, 0, cb, n->e[l], 1,
                              l < L - 1 ? n->a[l + 1] : nullptr);
    if (l < L - 1) {
      const int64_t cnt = (int64_t)(Hl / 2) * (Wl / 2) * n->ch[l];
      if (!pooled)
        k_pool2<<<grid_for(cnt), 256, 0, n->stream>>>(Hl / 2, Wl / 2, n->ch[l], n->e[l], n->a[l + 1], n->skip);
      a = n->a[l + 1];
      cprev = n->ch[l];
    }
  }
  const uint16_t* dnext = n->e[L - 1];
  for (int l = L - 2; l >= 0; --l) {
    const int Hl = H >> l, Wl = W >> l;
    const ConvLayer& ca = n->conv[conv_index(n, 'd', l, 0)];
    const ConvLayer& cb = n->conv[conv_index(n, 'd', l, 1)];
    conv3(n, Hl, Wl, dnext, n->ch[l + 1], 1, n->e[l], n->ch[l], ca, n->hd[l], 1);
    conv3(n, Hl, Wl, n->hd[l], n->ch[l], 0, nullptr, 0, cb, n->d[l], 1);
    dnext = n->d[l];
  }
  const int64_t npix = (int64_t)H * W;
  if (n->cout <= 4)
    k_head_fwd<4><<<grid_for(npix), 256, 0, n->stream>>>(npix, head_input(n), n->ch[0], n->P + n->head_w,
                                                         n->P + n->head_b, n->cout, n->y, n->skip);
  else
    k_head_fwd<16><<<grid_for(npix), 256, 0, n->stream>>>(npix, head_input(n), n->ch[0], n->P + n->head_w,
                                                          n->P + n->head_b, n->cout, n->y, n->skip);
}

// backward of o = relu(conv3(x)) given g = dL/do (FP32, H x W x cout):
// weight/bias gradients into G, input gradient (before any ReLU of x) into gx
void conv_layer_backward(m1nn* n, int H, int W, const float* g, const uint16_t* o, const uint16_t* x0, int C0,
                         int up0, const uint16_t* x1, int C1, const ConvLayer& c, float* gx) {
  const int64_t HW = (int64_t)H * W;
  if (wgrad_k32(W)) {
    const unsigned tiles = (unsigned)((HW + kTrPix - 1) / kTrPix);
    k_relu_grad_t<<<dim3(tiles, (c.cout + kTrCh - 1) / kTrCh), 256, 0, n->stream>>>((int)HW, c.cout, g, o, n->gpre,
                                                                                    n->gT);
    k_to_chw3<<<dim3(tiles, (C0 + C1 + kTrCh - 1) / kTrCh), 256, 0, n->stream>>>(H, W, x0, C0, up0, x1, C1, n->xT);
  } else {
    k_relu_grad<<<grid_for(HW * c.cout), 256, 0, n->stream>>>(HW, c.cout, g, o, n->gpre, n->gT);
    k_to_chw<<<grid_for(HW * (C0 + C1)), 256, 0, n->stream>>>(H, W, x0, C0, up0, x1, C1, n->xT);
  }
  conv3_wgrad(n, H, W, c);
  if (gx) conv3_dgrad(n, H, W, n->gpre, c, gx);
}

void backward_impl(m1nn* n, int H, int W) {
  const int L = n->L;
  const int64_t npix = (int64_t)H * W;
  // head
  {
    // head_b follows head_w in the slab: one sum over the partials writes both
    const int ppb = head_ppb(npix);
    const int nblk = (int)((npix + ppb - 1) / ppb);
    const dim3 grd(nblk, n->ch[0] / 8);
    if (n->cout <= 4)
      k_head_dw_part<4><<<grd, 256, 0, n->stream>>>(npix, ppb, n->gy, n->cout, head_input(n), n->ch[0], n->wpart);
    else
      k_head_dw_part<16><<<grd, 256, 0, n->stream>>>(npix, ppb, n->gy, n->cout, head_input(n), n->ch[0], n->wpart);
    const int64_t nh = (int64_t)n->cout * n->ch[0] + n->cout;
    k_sum_chunks<<<sum_grid(nh), 256, 0, n->stream>>>(n->wpart, nblk, nh, n->G + n->head_w);
  }
  float* gd = n->gbuf0;  // gradient w.r.t. d_l (FP32)
  k_head_dx<<<grid_for(npix * n->ch[0]), 256, 0, n->stream>>>(npix, n->gy, n->cout, n->P + n->head_w, n->ch[0], gd);
  // decoder, level 0 upward
  for (int l = 0; l < L - 1; ++l) {
    const int Hl = H >> l, Wl = W >> l;
    const ConvLayer& ca = n->conv[conv_index(n, 'd', l, 0)];
    const ConvLayer& cb = n->conv[conv_index(n, 'd', l, 1)];
    float* gh = n->gbuf1;
    conv_layer_backward(n, Hl, Wl, gd, n->d[l], n->hd[l], n->ch[l], 0, nullptr, 0, cb, gh);
    const uint16_t* dnext = (l + 1 == L - 1) ? n->e[L - 1] : n->d[l + 1];
    float* gcat = n->gbuf2;
    conv_layer_backward(n, Hl, Wl, gh, n->hd[l], dnext, n->ch[l + 1], 1, n->e[l], n->ch[l], ca, gcat);
    // split: gradient of d_{l+1} (half resolution) and of the skip e_l
    float* gdn = n->gbuf0;
    const int64_t cnt = (int64_t)(Hl / 2) * (Wl / 2) * n->ch[l + 1] + (int64_t)Hl * Wl * n->ch[l];
    k_split_cat<<<grid_for(cnt), 256, 0, n->stream>>>(Hl, Wl, n->ch[l + 1], n->ch[l], gcat, gdn, n->genc[l]);
    gd = gdn;
  }
  // bottom: d_{L-1} = e_{L-1}
  float* ge = n->gbuf1;
  hipMemcpyAsync(ge, gd, sizeof(float) * (size_t)((H >> (L - 1)) * (W >> (L - 1)) * n->ch[L - 1]),
                 hipMemcpyDeviceToDevice, n->stream);
  for (int l = L - 1; l >= 0; --l) {
    const int Hl = H >> l, Wl = W >> l;
    const ConvLayer& ca = n->conv[conv_index(n, 'e', l, 0)];
    const ConvLayer& cb = n->conv[conv_index(n, 'e', l, 1)];
    float* gh = n->gbuf2;
    conv_layer_backward(n, Hl, Wl, ge, n->e[l], n->ha[l], n->ch[l], 0, nullptr, 0, cb, gh);
    const uint16_t* xin = l == 0 ? n->in : n->a[l];
    const int cin = l == 0 ? n->cin_pad : n->ch[l - 1];
    float* ga = l == 0 ? nullptr : n->gbuf0;
    conv_layer_backward(n, Hl, Wl, gh, n->ha[l], xin, cin, 0, nullptr, 0, ca, ga);
    if (l > 0) {
      // gradient of e_{l-1} = skip gradient + average-pool backward of ga
      const int Hp = H >> (l - 1), Wp = W >> (l - 1);
      float* gen = n->gbuf1;
      const int64_t cnt = (int64_t)Hp * Wp * n->ch[l - 1];
      k_pool_back_add<<<grid_for(cnt), 256, 0, n->stream>>>(Hp, Wp, n->ch[l - 1], ga, n->genc[l - 1], gen);
      ge = gen;
    }
  }
}

m1_status check_size(m1nn* n, int H, int W) {
  const int q = 1 << (n->L - 1);
  if (H < q || W < q || H % q || W % q || H > n->Hmax || W > n->Wmax) {
    n->err = "H and W must be multiples of 2^(levels-1) and not exceed the sizes given at creation";
    return M1_ERR_INVALID_ARG;
  }
  return M1_OK;
}

}  // namespace

// ============================================================================
// C ABI (network)
// ============================================================================
extern "C" {

m1_status m1nn_create(int32_t cin, int32_t cout, int32_t levels, const int32_t* channels, int32_t Hmax, int32_t Wmax,
                      void* hip_stream, m1nn** out) {
  if (!out) return M1_ERR_INVALID_ARG;
  *out = nullptr;
  if (cin < 1 || cin > 64 || cout < 1 || cout > 16 || levels < 1 || levels > 6 || !channels || Hmax < 1 || Wmax < 1)
    return M1_ERR_INVALID_ARG;
  for (int l = 0; l < levels; ++l)
    if (channels[l] < 16 || channels[l] > 256 || channels[l] % 16) return M1_ERR_INVALID_ARG;
  const int q = 1 << (levels - 1);
  if (Hmax % q || Wmax % q) return M1_ERR_INVALID_ARG;
  m1nn* n = new m1nn();
  n->cin = cin;
  n->cin_pad = (cin + 15) / 16 * 16;
  n->cout = cout;
  n->L = levels;
  for (int l = 0; l < levels; ++l) n->ch[l] = channels[l];
  n->Hmax = Hmax;
  n->Wmax = Wmax;
  n->stream = (hipStream_t)hip_stream;
  // layer table and parameter slab (padded layout)
  int64_t off = 0;
  auto add = [&](int ci_pad, int ci_true, int co) {
    ConvLayer c;
    c.cin = ci_pad;
    c.cin_true = ci_true;
    c.cout = co;
    c.woff = off;
    c.wsize = (int64_t)9 * co * ci_pad;
    off += c.wsize;
    c.boff = off;
    off += co;
    n->conv.push_back(c);
  };
  int prev = n->cin_pad, prev_true = cin;
  for (int l = 0; l < levels; ++l) {
    add(prev, prev_true, channels[l]);
    add(channels[l], channels[l], channels[l]);
    prev = prev_true = channels[l];
  }
  for (int l = levels - 2; l >= 0; --l) {
    add(channels[l + 1] + channels[l], channels[l + 1] + channels[l], channels[l]);
    add(channels[l], channels[l], channels[l]);
  }
  n->head_w = off;
  off += (int64_t)cout * channels[0];
  n->head_b = off;
  off += cout;
  n->nparam = off;
  bool good = alloc(n, &n->P, off) && alloc(n, &n->G, off) && alloc(n, &n->Mo, off) && alloc(n, &n->Vo, off);
  for (auto& c : n->conv) good = good && alloc(n, &c.wf, c.wsize) && alloc(n, &c.wt, c.wsize);
  const int64_t HW = (int64_t)Hmax * Wmax;
  int cmax = n->cin_pad;
  for (int l = 0; l < levels; ++l) cmax = std::max(cmax, channels[l] + (l + 1 < levels ? channels[l + 1] : 0));
  good = good && alloc(n, &n->in, HW * n->cin_pad) && alloc(n, &n->y, HW * cout) && alloc(n, &n->gy, HW * cout);
  n->ha.assign(levels, nullptr);
  n->e.assign(levels, nullptr);
  n->a.assign(levels, nullptr);
  n->hd.assign(levels, nullptr);
  n->d.assign(levels, nullptr);
  n->genc.assign(levels, nullptr);
  for (int l = 0; l < levels && good; ++l) {
    const int64_t hw = HW >> (2 * l);
    good = alloc(n, &n->ha[l], hw * channels[l]) && alloc(n, &n->e[l], hw * channels[l]) &&
           alloc(n, &n->genc[l], hw * channels[l]);
    if (good && l > 0) good = alloc(n, &n->a[l], hw * channels[l - 1]);
    if (good && l < levels - 1) good = alloc(n, &n->hd[l], hw * channels[l]) && alloc(n, &n->d[l], hw * channels[l]);
  }
  good = good && alloc(n, &n->gbuf0, HW * cmax) && alloc(n, &n->gbuf1, HW * cmax) && alloc(n, &n->gbuf2, HW * cmax) &&
         alloc(n, &n->gpre, HW * cmax) && alloc(n, &n->xT, 3 * HW * cmax) && alloc(n, &n->gT, HW * cmax);
  // partial sums: the K = 32 weight gradient takes at most max(1, kWgradBlocks / blocks)
  // chunks, the other one ceil(HW / 4096), the head at most 256 blocks
  int64_t wlen = 256 * ((int64_t)cout * channels[0] + cout), blen = 0;
  for (auto& c : n->conv) {
    const int64_t blocks = ((c.cout + 63) / 64) * ((c.cin + 15) / 16);
    const int64_t nk32 = std::max<int64_t>(1, kWgradBlocks / blocks);
    wlen = std::max(wlen, c.wsize * std::max(nk32, (HW + 4095) / 4096));
    blen = std::max(blen, (int64_t)c.cout * nk32);
  }
  n->wpart_len = wlen;
  good = good && alloc(n, &n->wpart, n->wpart_len) && alloc(n, &n->bpart, blen) &&
         alloc(n, &n->loss_part, 2 * 1024) && alloc(n, &n->loss_out, 2);
  if (!good) {
    nn_free(n);
    delete n;
    return M1_ERR_OUT_OF_MEMORY;
  }
  hipMemsetAsync(n->P, 0, sizeof(float) * off, n->stream);
  hipMemsetAsync(n->G, 0, sizeof(float) * off, n->stream);
  hipMemsetAsync(n->Mo, 0, sizeof(float) * off, n->stream);
  hipMemsetAsync(n->Vo, 0, sizeof(float) * off, n->stream);
  refresh_weights(n);
  if (hipStreamSynchronize(n->stream) != hipSuccess) {
    nn_free(n);
    delete n;
    return M1_ERR_HIP;
  }
  *out = n;
  return M1_OK;
}

int64_t m1nn_param_count(const m1nn* n) {
  if (!n) return 0;
  int64_t cnt = 0;
  for (auto& c : n->conv) cnt += (int64_t)9 * c.cin_true * c.cout + c.cout;
  return cnt + (int64_t)n->cout * n->ch[0] + n->cout;
}

// Host copy of the parameters in definition order, each conv3 weight as
// [dy][dx][ci][co] (unpadded) then its bias; the head as [ci][co] then bias.
static m1_status copy_params(m1nn* n, float* host, int64_t count, bool to_device, bool grads) {
  if (!n || !host) return M1_ERR_INVALID_ARG;
  if (count != m1nn_param_count(n)) { n->err = "parameter count mismatch"; return M1_ERR_INVALID_ARG; }
  std::vector<float> slab(n->nparam, 0.f);
  const float* src = grads ? n->G : n->P;
  if (!ok(n, hipMemcpyAsync(slab.data(), src, sizeof(float) * n->nparam, hipMemcpyDeviceToHost, n->stream), "copy") ||
      !ok(n, hipStreamSynchronize(n->stream), "sync"))
    return M1_ERR_HIP;
  int64_t k = 0;
  for (auto& c : n->conv) {
    for (int tap = 0; tap < 9; ++tap)
      for (int ci = 0; ci < c.cin_true; ++ci)
        for (int co = 0; co < c.cout; ++co) {
          float& s = slab[c.woff + ((int64_t)tap * c.cout + co) * c.cin + ci];
          if (to_device) s = host[k++]; else host[k++] = s;
        }
    for (int co = 0; co < c.cout; ++co) {
      float& s = slab[c.boff + co];
      if (to_device) s = host[k++]; else host[k++] = s;
    }
  }
  for (int ci = 0; ci < n->ch[0]; ++ci)
    for (int co = 0; co < n->cout; ++co) {
      float& s = slab[n->head_w + (int64_t)co * n->ch[0] + ci];
      if (to_device) s = host[k++]; else host[k++] = s;
    }
  for (int co = 0; co < n->cout; ++co) {
    float& s = slab[n->head_b + co];
    if (to_device) s = host[k++]; else host[k++] = s;
  }
  if (to_device) {
    if (!ok(n, hipMemcpyAsync(n->P, slab.data(), sizeof(float) * n->nparam, hipMemcpyHostToDevice, n->stream), "copy"))
      return M1_ERR_HIP;
    refresh_weights(n);
    if (!ok(n, hipStreamSynchronize(n->stream), "sync")) return M1_ERR_HIP;
  }
  return M1_OK;
}

m1_status m1nn_set_params(m1nn* n, const float* host, int64_t count) {
  return copy_params(n, const_cast<float*>(host), count, true, false);
}
m1_status m1nn_get_params(m1nn* n, float* host, int64_t count) { return copy_params(n, host, count, false, false); }
m1_status m1nn_get_grads(m1nn* n, float* host, int64_t count) { return copy_params(n, host, count, false, true); }

// He-normal initial weights (He et al. 2015: N(0, 2/fan_in) with fan_in = 9 C_in for a 3x3
// convolution), zero biases, the 1x1 head N(0, 1/C) scaled by head_scale.  Normal draws:
// SplitMix64 (Steele, Lea & Flood 2014) on the counter seed*2^32 + k gives two 53-bit
// uniforms per pair, mapped by the Box-Muller transform; parameters are visited in the
// definition order of m1nn_set_params, so a given seed always gives the same weights.
m1_status m1nn_init_params(m1nn* n, uint64_t seed, float head_scale) {
  if (!n || !std::isfinite(head_scale)) return M1_ERR_INVALID_ARG;
  uint64_t ctr = seed << 32;
  auto splitmix = [&]() {
    uint64_t z = (ctr += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  bool have = false;
  double spare = 0.0;
  auto normal = [&]() {
    if (have) { have = false; return spare; }
    const double u1 = ((splitmix() >> 11) + 1.0) * 0x1.0p-53;   // (0, 1]
    const double u2 = (splitmix() >> 11) * 0x1.0p-53;           // [0, 1)
    const double rad = std::sqrt(-2.0 * std::log(u1));
    const double ang = 6.283185307179586477 * u2;
    spare = rad * std::sin(ang);
    have = true;
    return rad * std::cos(ang);
  };
  const int64_t cnt = m1nn_param_count(n);
  std::vector<float> h(cnt, 0.f);
  int64_t k = 0;
  for (auto& c : n->conv) {
    const double sd = std::sqrt(2.0 / (9.0 * c.cin_true));
    const int64_t nw = (int64_t)9 * c.cin_true * c.cout;
    for (int64_t i = 0; i < nw; ++i) h[k++] = (float)(sd * normal());
    k += c.cout;   // biases stay 0
  }
  const double sdh = std::sqrt(1.0 / n->ch[0]) * head_scale;
  for (int64_t i = 0; i < (int64_t)n->ch[0] * n->cout; ++i) h[k++] = (float)(sdh * normal());
  k += n->cout;
  if (k != cnt) { n->err = "parameter layout mismatch"; return M1_ERR_INVALID_ARG; }
  return m1nn_set_params(n, h.data(), cnt);
}

m1_status m1nn_forward(m1nn* n, const float* x, int32_t H, int32_t W, float* y) {
  if (!n || !x || !y) return M1_ERR_INVALID_ARG;
  m1_status st = check_size(n, H, W);
  if (st != M1_OK) return st;
  const int64_t npix = (int64_t)H * W;
  k_pack<<<grid_for(npix * n->cin_pad), 256, 0, n->stream>>>(npix, x, n->cin, n->cin_pad, n->in);
  forward_impl(n, H, W);
  if (!ok(n, hipMemcpyAsync(y, n->y, sizeof(float) * npix * n->cout, hipMemcpyDeviceToDevice, n->stream), "copy"))
    return M1_ERR_HIP;
  return ok(n, hipGetLastError(), "launch") ? M1_OK : M1_ERR_HIP;
}

m1_status m1nn_backward(m1nn* n, const float* x, const float* target, int32_t H, int32_t W, double* loss) {
  if (!n || !x || !target) return M1_ERR_INVALID_ARG;
  m1_status st = check_size(n, H, W);
  if (st != M1_OK) return st;
  const int64_t npix = (int64_t)H * W;
  const int64_t ny = npix * n->cout;
  k_pack<<<grid_for(npix * n->cin_pad), 256, 0, n->stream>>>(npix, x, n->cin, n->cin_pad, n->in);
  forward_impl(n, H, W);
  const int nb = (int)std::min<int64_t>(1024, (ny + 255) / 256);
  k_loss_part<<<nb, 256, 0, n->stream>>>(ny, n->y, target, n->loss_part);
  k_loss_final<<<1, 256, 0, n->stream>>>(n->loss_part, nb, n->loss_out);
  k_loss_grad<<<grid_for(ny), 256, 0, n->stream>>>(ny, n->y, target, n->loss_out, n->gy);
  backward_impl(n, H, W);
  double lh[2] = {0, 0};
  if (!ok(n, hipMemcpyAsync(lh, n->loss_out, sizeof(lh), hipMemcpyDeviceToHost, n->stream), "copy") ||
      !ok(n, hipStreamSynchronize(n->stream), "sync"))
    return M1_ERR_HIP;
  if (loss) *loss = lh[0];
  return std::isfinite(lh[0]) ? M1_OK : M1_ERR_NONFINITE;
}

m1_status m1nn_adam_step(m1nn* n, float lr) {
  if (!n || !(lr > 0)) return M1_ERR_INVALID_ARG;
  n->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)n->adam_t), c2 = 1.f - std::pow(b2, (float)n->adam_t);
  k_adam<<<grid_for(n->nparam), 256, 0, n->stream>>>(n->nparam, n->P, n->G, n->Mo, n->Vo, lr, b1, b2, 1e-8f, c1, c2);
  refresh_weights(n);
  return ok(n, hipGetLastError(), "launch") ? M1_OK : M1_ERR_HIP;
}

m1_status m1nn_train_step(m1nn* n, const float* x, const float* target, int32_t H, int32_t W, float lr, double* loss) {
  m1_status st = m1nn_backward(n, x, target, H, W, loss);
  if (st != M1_OK) return st;
  return m1nn_adam_step(n, lr);
}

m1_status m1nn_save(m1nn* n, const char* path) {
  if (!n || !path) return M1_ERR_INVALID_ARG;
  const int64_t cnt = m1nn_param_count(n);
  std::vector<float> h(cnt);
  m1_status st = m1nn_get_params(n, h.data(), cnt);
  if (st != M1_OK) return st;
  FILE* f = std::fopen(path, "wb");
  if (!f) { n->err = "cannot open file"; return M1_ERR_INVALID_ARG; }
  const int32_t head[4 + 8] = {0x4D314E4E, n->cin, n->cout, n->L, n->ch[0], n->ch[1], n->ch[2], n->ch[3],
                               n->ch[4], n->ch[5], n->ch[6], n->ch[7]};
  bool good = std::fwrite(head, sizeof(head), 1, f) == 1 && std::fwrite(h.data(), sizeof(float), cnt, f) == (size_t)cnt;
  std::fclose(f);
  return good ? M1_OK : M1_ERR_INVALID_ARG;
}

m1_status m1nn_load(m1nn* n, const char* path) {
  if (!n || !path) return M1_ERR_INVALID_ARG;
  FILE* f = std::fopen(path, "rb");
  if (!f) { n->err = "cannot open file"; return M1_ERR_INVALID_ARG; }
  int32_t head[12];
  bool good = std::fread(head, sizeof(head), 1, f) == 1 && head[0] == 0x4D314E4E && head[1] == n->cin &&
              head[2] == n->cout && head[3] == n->L;
  for (int l = 0; l < n->L && good; ++l) good = head[4 + l] == n->ch[l];
  const int64_t cnt = m1nn_param_count(n);
  std::vector<float> h(cnt);
  good = good && std::fread(h.data(), sizeof(float), cnt, f) == (size_t)cnt;
  std::fclose(f);
  if (!good) { n->err = "weight file does not match this network"; return M1_ERR_INVALID_ARG; }
  return m1nn_set_params(n, h.data(), cnt);
}

void m1nn_destroy(m1nn* n) {
  if (!n) return;
  if (n->stream) hipStreamSynchronize(n->stream);
  nn_free(n);
  delete n;
}

const char* m1nn_last_error(const m1nn* n) { return n ? n->err.c_str() : ""; }

}  // extern "C"

namespace m1 {
// device pointers used by the learned preconditioner inside GMRES
uint16_t* nn_input(m1nn* n) { return n->in; }
const float* nn_output(m1nn* n) { return n->y; }
int nn_cin_pad(const m1nn* n) { return n->cin_pad; }
int nn_cin(const m1nn* n) { return n->cin; }
int nn_cout(const m1nn* n) { return n->cout; }
m1_status nn_run(m1nn* n, int H, int W, hipStream_t s, const int* skip) {
  m1_status st = check_size(n, H, W);
  if (st != M1_OK) return st;
  hipStream_t keep = n->stream;
  n->stream = s;
  n->skip = skip;
  forward_impl(n, H, W);
  n->stream = keep;
  n->skip = nullptr;
  return M1_OK;
}
int nn_levels(const m1nn* n) { return n->L; }
int nn_hmax(const m1nn* n) { return n->Hmax; }
int nn_wmax(const m1nn* n) { return n->Wmax; }
}  // namespace m1

namespace m1 {

constexpr int kNnCin = 9;

template <typename TV>
__global__ void k_nn_features(int64_t N, const TV* __restrict__ r, const double* __restrict__ rnorm2,
                              const double* __restrict__ bjinv, const double* __restrict__ Uk,
                              const double* __restrict__ sigma, double c, double cdt, int cpad,
                              uint16_t* __restrict__ in_bf16, float* __restrict__ out_f32,
                              const int* __restrict__ skip) {
  if (skip && *skip) return;
  const double rn = sqrt(fmax(rnorm2[0], 0.0));
  const double sc = rn > 0 ? sqrt(3.0 * (double)N) / rn : 0.0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
    double rv[3], f[kNnCin];
    for (int k = 0; k < 3; ++k) rv[k] = (double)r[k * N + p];
    for (int k = 0; k < 3; ++k) {
      f[k] = sc * rv[k];
      double z = 0.0;
      for (int q = 0; q < 3; ++q) z += bjinv[(k * 3 + q) * N + p] * rv[q];
      f[3 + k] = sc * z;
    }
    f[6] = log10(1.0 + sigma[p] * cdt) * 0.25;
    const double E = Uk[p], Fx = Uk[N + p], Fy = Uk[2 * N + p];
    const double Fm = sqrt(Fx * Fx + Fy * Fy);
    const double fr = Fm / (c * fmax(E, 1e-300));
    const double scale = fr > 1.0 ? 1.0 / fr : 1.0;
    f[7] = Fx / (c * fmax(E, 1e-300)) * scale;
    f[8] = Fy / (c * fmax(E, 1e-300)) * scale;
    if (in_bf16) {
      for (int k = 0; k < cpad; ++k) in_bf16[p * cpad + k] = k < kNnCin ? f2bf((float)f[k]) : (uint16_t)0;
    }
    if (out_f32) {
      for (int k = 0; k < kNnCin; ++k) out_f32[p * kNnCin + k] = (float)f[k];
    }
  }
}

template <typename TV>
void launch_nn_features(int64_t N, const TV* r, const double* rnorm2, const double* bjinv, const double* Uk,
                        const double* sigma, double c, double cdt, int cpad, uint16_t* in_bf16, float* out_f32,
                        hipStream_t s, const int* skip) {
  k_nn_features<TV><<<grid_for(N), 256, 0, s>>>(N, r, rnorm2, bjinv, Uk, sigma, c, cdt, cpad, in_bf16, out_f32,
                                                skip);
}

template <typename TV, typename TZ>
__global__ void k_nn_combine(int64_t N, const TV* __restrict__ r, const double* __restrict__ rnorm2,
                             const double* __restrict__ bjinv, const float* __restrict__ y, TZ* __restrict__ z,
                             const int* __restrict__ skip) {
  if (skip && *skip) return;
  const double rn = sqrt(fmax(rnorm2[0], 0.0));
  const double back = rn / sqrt(3.0 * (double)N);
  // z = M^{-1} (r + (|r|/s) y): the network corrects the residual, block-Jacobi maps
  // the corrected residual to each cell's own scale
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
    double rv[3];
    for (int k = 0; k < 3; ++k) rv[k] = (double)r[k * N + p] + back * (double)y[p * 3 + k];
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int q = 0; q < 3; ++q) acc += bjinv[(k * 3 + q) * N + p] * rv[q];
      z[k * N + p] = (TZ)acc;
    }
  }
}

template <typename TV, typename TZ>
void launch_nn_combine(int64_t N, const TV* r, const double* rnorm2, const double* bjinv, const float* y, TZ* z,
                       hipStream_t s, const int* skip) {
  k_nn_combine<TV, TZ><<<grid_for(N), 256, 0, s>>>(N, r, rnorm2, bjinv, y, z, skip);
}

__global__ void k_nn_target(int64_t N, const double* __restrict__ r, const double* __restrict__ e,
                            const double* __restrict__ rnorm2, const double* __restrict__ bjinv,
                            float* __restrict__ t) {
  const double rn = sqrt(fmax(rnorm2[0], 0.0));
  const double sc = rn > 0 ? sqrt(3.0 * (double)N) / rn : 0.0;
  // t = s (M e - r)/|r| with M the diagonal block (the inverse of the stored inverse,
  // by cofactors): the residual correction that M^{-1} maps onto the error e
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
    double B[3][3];
    for (int k = 0; k < 3; ++k)
      for (int q = 0; q < 3; ++q) B[k][q] = bjinv[(k * 3 + q) * N + p];
    const double c00 = B[1][1] * B[2][2] - B[1][2] * B[2][1];
    const double c01 = B[1][2] * B[2][0] - B[1][0] * B[2][2];
    const double c02 = B[1][0] * B[2][1] - B[1][1] * B[2][0];
    const double det = B[0][0] * c00 + B[0][1] * c01 + B[0][2] * c02;
    double M[3][3];
    M[0][0] = c00;
    M[1][0] = c01;
    M[2][0] = c02;
    M[0][1] = B[0][2] * B[2][1] - B[0][1] * B[2][2];
    M[1][1] = B[0][0] * B[2][2] - B[0][2] * B[2][0];
    M[2][1] = B[0][1] * B[2][0] - B[0][0] * B[2][1];
    M[0][2] = B[0][1] * B[1][2] - B[0][2] * B[1][1];
    M[1][2] = B[0][2] * B[1][0] - B[0][0] * B[1][2];
    M[2][2] = B[0][0] * B[1][1] - B[0][1] * B[1][0];
    const double idet = 1.0 / det;
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int q = 0; q < 3; ++q) acc += M[k][q] * idet * e[q * N + p];
      t[p * 3 + k] = (float)(sc * (acc - r[k * N + p]));
    }
  }
}

void launch_nn_target(int64_t N, const double* r, const double* e, const double* rnorm2, const double* bjinv,
                      float* t, hipStream_t s) {
  k_nn_target<<<grid_for(N), 256, 0, s>>>(N, r, e, rnorm2, bjinv, t);
}

template void launch_nn_features<double>(int64_t, const double*, const double*, const double*, const double*,
                                         const double*, double, double, int, uint16_t*, float*, hipStream_t,
                                         const int*);
template void launch_nn_features<float>(int64_t, const float*, const double*, const double*, const double*,
                                        const double*, double, double, int, uint16_t*, float*, hipStream_t,
                                         const int*);
template void launch_nn_combine<double, double>(int64_t, const double*, const double*, const double*, const float*,
                                                double*, hipStream_t, const int*);
template void launch_nn_combine<float, float>(int64_t, const float*, const double*, const double*, const float*,
                                              float*, hipStream_t, const int*);
template void launch_nn_combine<double, float>(int64_t, const double*, const double*, const double*, const float*,
                                               float*, hipStream_t, const int*);

}  // namespace m1
