// Device helpers shared by the inference and training kernels: block-centre grid sampling, bilinear
// blend, float -> bfloat16 rounding, and the BC packing of one texture of one block position.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntbc.h"

namespace ntbc {
namespace dev {

// Grid sampling (paper Sec. 3.1 / Sec. 3.4: grids indexed by the normalised block coordinate).  Block b
// of a grid of `blocks` blocks samples a level of `res` vertices at p = (b + 1/2) res / blocks - 1/2,
// clamped to [0, res-1]: p = num / (2 blocks) with num = (2b + 1) res - blocks, so the lower corner
// i0 = min(floor(p), res-2) is an integer decision and the fraction f = fnum / (2 blocks) is exact
// whenever 2*blocks is a power of two.
struct Corner {
  int i0;
  float f;
};

__device__ __forceinline__ Corner corner(int b, int blocks, int res) {
  const int64_t den = 2 * (int64_t)blocks;
  const int64_t num = (int64_t)(2 * b + 1) * res - blocks;
  Corner c;
  if (num <= 0) {
    c.i0 = 0;
    c.f = 0.0f;
  } else if (num >= (int64_t)(res - 1) * den) {
    c.i0 = res - 2;
    c.f = 1.0f;
  } else {
    c.i0 = (int)(num / den);
    c.f = (float)(num - (int64_t)c.i0 * den) / (float)den;
  }
  return c;
}

// Round-to-nearest-even float -> bfloat16 bits (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  return bf16_bits(lo) | (bf16_bits(hi) << 16);
}

// Loads FE consecutive features of one grid vertex and returns them as floats (real values).
template <int FE>
__device__ __forceinline__ void load_u8(const uint8_t* p, float v[FE]) {
  if constexpr (FE == 8) {
    const uint2 w = *reinterpret_cast<const uint2*>(p);
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = (float)((w.x >> (8 * m)) & 0xFF);
#pragma unroll
    for (int m = 0; m < 4; ++m) v[4 + m] = (float)((w.y >> (8 * m)) & 0xFF);
  } else if constexpr (FE == 4) {
    const uint32_t w = *reinterpret_cast<const uint32_t*>(p);
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] = (float)((w >> (8 * m)) & 0xFF);
  } else {
#pragma unroll
    for (int m = 0; m < FE; ++m) v[m] = (float)p[m];
  }
}

template <int FE>
__device__ __forceinline__ void load_f32(const float* p, float v[FE]) {
  if constexpr (FE % 4 == 0) {
#pragma unroll
    for (int m = 0; m < FE; m += 4) {
      const float4 q = *reinterpret_cast<const float4*>(p + m);
      v[m] = q.x;
      v[m + 1] = q.y;
      v[m + 2] = q.z;
      v[m + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int m = 0; m < FE; ++m) v[m] = p[m];
  }
}

struct GridView {
  const uint8_t* u8;     // U8 codes, or
  const float* f32;      // real values
  const float* scale;    // per level (U8)
  const int32_t* zero;   // per level (U8)
  int n_levels, base_res, n_features, blocks_w, blocks_h;
  // shift_x = log2(2*blocks_w) when that is a power of two and every numerator fits in 31 bits,
  // else -1 (general path); likewise shift_y
  int shift_x, shift_y;
  // fast8: uint8 grid, 8 features per vertex, both shifts >= 0 and every byte offset below 2^31
  // (sample8_fast: 32-bit offsets from the grid base)
  int fast8;
  int64_t level_offset[NTBC_MAX_LEVELS + 1];
};

// corner() when 2*blocks = 2^shift: the same integer decisions with shifts instead of divisions.
__device__ __forceinline__ Corner corner_pow2(int b, int blocks, int res, int shift) {
  const int num = (2 * b + 1) * res - blocks;
  const int hi = (res - 1) << shift;
  const int i0 = num >> shift;
  Corner c;
  c.i0 = num <= 0 ? 0 : (num >= hi ? res - 2 : i0);
  const int fnum = num <= 0 ? 0 : (num >= hi ? (1 << shift) : num - (i0 << shift));
  c.f = (float)fnum * __int_as_float((127 - shift) << 23);  // exact: 2^-shift
  return c;
}

// Bilinear feature values of features [f0, f0+FE) of `level` at block (bx, by):
// sum over the four corners of w_c * value_c, value = scale*(q - zero) for U8 grids.
template <int FE>
__device__ __forceinline__ void sample(const GridView& g, int level, int f0, int bx, int by, float out[FE]) {
  const int res = g.base_res << level;
  const Corner cx = g.shift_x >= 0 ? corner_pow2(bx, g.blocks_w, res, g.shift_x) : corner(bx, g.blocks_w, res);
  const Corner cy = g.shift_y >= 0 ? corner_pow2(by, g.blocks_h, res, g.shift_y) : corner(by, g.blocks_h, res);
  const int64_t v00 = g.level_offset[level] + (int64_t)cy.i0 * res + cx.i0;
  const int64_t F = g.n_features;
  const float w00 = (1.0f - cx.f) * (1.0f - cy.f), w10 = cx.f * (1.0f - cy.f);
  const float w01 = (1.0f - cx.f) * cy.f, w11 = cx.f * cy.f;
  float a[FE], b[FE], c[FE], d[FE];
  if (g.u8) {
    load_u8<FE>(g.u8 + v00 * F + f0, a);
    load_u8<FE>(g.u8 + (v00 + 1) * F + f0, b);
    load_u8<FE>(g.u8 + (v00 + res) * F + f0, c);
    load_u8<FE>(g.u8 + (v00 + res + 1) * F + f0, d);
    const float s = g.scale[level];
    const float sz = -s * (float)g.zero[level];
#pragma unroll
    for (int m = 0; m < FE; ++m) out[m] = fmaf(s, fmaf(w00, a[m], fmaf(w10, b[m], fmaf(w01, c[m], w11 * d[m]))), sz);
  } else {
    load_f32<FE>(g.f32 + v00 * F + f0, a);
    load_f32<FE>(g.f32 + (v00 + 1) * F + f0, b);
    load_f32<FE>(g.f32 + (v00 + res) * F + f0, c);
    load_f32<FE>(g.f32 + (v00 + res + 1) * F + f0, d);
#pragma unroll
    for (int m = 0; m < FE; ++m) out[m] = fmaf(w00, a[m], fmaf(w10, b[m], fmaf(w01, c[m], w11 * d[m])));
  }
}

// sample<8> for a fast8 grid: the same corners and blend, with 32-bit byte offsets from the grid base
// (a scalar base plus a per-lane offset in the loads instead of 64-bit per-lane addresses).
__device__ __forceinline__ void sample8_fast(const GridView& g, int level, int bx, int by, float out[8]) {
  const int res = g.base_res << level;
  const Corner cx = corner_pow2(bx, g.blocks_w, res, g.shift_x);
  const Corner cy = corner_pow2(by, g.blocks_h, res, g.shift_y);
  const uint32_t o00 = ((uint32_t)g.level_offset[level] + (uint32_t)(cy.i0 * res + cx.i0)) * 8u;
  const uint32_t row = 8u * (uint32_t)res;
  const float w00 = (1.0f - cx.f) * (1.0f - cy.f), w10 = cx.f * (1.0f - cy.f);
  const float w01 = (1.0f - cx.f) * cy.f, w11 = cx.f * cy.f;
  float a[8], b[8], c[8], d[8];
  load_u8<8>(g.u8 + o00, a);
  load_u8<8>(g.u8 + (o00 + 8u), b);
  load_u8<8>(g.u8 + (o00 + row), c);
  load_u8<8>(g.u8 + (o00 + row + 8u), d);
  const float s = g.scale[level];
  const float sz = -s * (float)g.zero[level];
#pragma unroll
  for (int m = 0; m < 8; ++m) out[m] = fmaf(s, fmaf(w00, a[m], fmaf(w10, b[m], fmaf(w01, c[m], w11 * d[m]))), sz);
}

// Input features c0 .. c0+NV-1 of the concatenation [level 0 features, level 1 features, ...], zero
// past in_dim.  NV is 8 (BF16/FP8 operands) or 1 (FP32 operands); n_features is 1, 2, 4, 8 or 16.
template <int NV>
__device__ __forceinline__ void features(const GridView& g, int c0, int bx, int by, float v[NV]) {
  const int in_dim = g.n_levels * g.n_features;
  if constexpr (NV == 1) {
    if (c0 < in_dim) {
      float t[1];
      sample<1>(g, c0 / g.n_features, c0 % g.n_features, bx, by, t);
      v[0] = t[0];
    } else {
      v[0] = 0.0f;
    }
  } else {
    static_assert(NV == 8, "feature groups of 8");
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = 0.0f;
    if (c0 >= in_dim) return;
    if (g.fast8) {
      sample8_fast(g, c0 / 8, bx, by, v);
      return;
    }
    switch (g.n_features) {
      case 16:
        sample<8>(g, c0 / 16, c0 % 16, bx, by, v);
        break;
      case 8:
        sample<8>(g, c0 / 8, 0, bx, by, v);
        break;
      case 4:
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (c0 + 4 * h < in_dim) sample<4>(g, c0 / 4 + h, 0, bx, by, v + 4 * h);
        break;
      case 2:
#pragma unroll
        for (int h = 0; h < 4; ++h)
          if (c0 + 2 * h < in_dim) sample<2>(g, c0 / 2 + h, 0, bx, by, v + 2 * h);
        break;
      default:
#pragma unroll
        for (int h = 0; h < 8; ++h)
          if (c0 + h < in_dim) sample<1>(g, c0 + h, 0, bx, by, v + h);
        break;
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Heads -> BC words (paper Sec. 3.2, Eq. palette, Eq. dist).  Decisions are taken in float32 with
// uncontracted operations: q = floor(y*(2^b-1) + 0.5) clamped; palette entry = code/255; squared
// distance ((d0*d0 + d1*d1) + d2*d2); first minimum in weight order.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ int quant_bits(float y, float mx) {
  float t = floorf(__fadd_rn(__fmul_rn(y, mx), 0.5f));
  t = fminf(fmaxf(t, 0.0f), mx);
  return (int)t;
}

__device__ __forceinline__ int expand5d(int v) { return (v << 3) | (v >> 2); }
__device__ __forceinline__ int expand6d(int v) { return (v << 2) | (v >> 4); }

struct Bc1Pal {
  uint32_t c0, c1;
  uint32_t map;     // stored 2-bit code of weight index n at bits 2n (0 for every texel when c0 == c1)
  float pal[4][3];  // weight order
};

// tab (optional): tab[c] = c / 255 as float32 (correctly rounded), replacing the division.
__device__ __forceinline__ float unit8(int c, const float* tab) { return tab ? tab[c] : (float)c / 255.0f; }

// Palette of two quantised RGB565 endpoints: the larger word becomes c0 (four-colour mode, Sec. 3),
// entries in weight order a, (2a+b)/3, (a+2b)/3, b of the expanded 8-bit channels.
__device__ __forceinline__ Bc1Pal bc1_palette(uint32_t c0, uint32_t c1, const float* tab = nullptr) {
  if (c0 < c1) {
    const uint32_t t = c0;
    c0 = c1;
    c1 = t;
  }
  Bc1Pal p;
  p.c0 = c0;
  p.c1 = c1;
  p.map = c0 == c1 ? 0u : 0x78u;  // weight order 0,1,2,3 -> codes 0,2,3,1
  const int a[3] = {expand5d((c0 >> 11) & 31), expand6d((c0 >> 5) & 63), expand5d(c0 & 31)};
  const int b[3] = {expand5d((c1 >> 11) & 31), expand6d((c1 >> 5) & 63), expand5d(c1 & 31)};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    p.pal[0][c] = unit8(a[c], tab);
    p.pal[1][c] = unit8((2 * a[c] + b[c] + 1) / 3, tab);
    p.pal[2][c] = unit8((a[c] + 2 * b[c] + 1) / 3, tab);
    p.pal[3][c] = unit8(b[c], tab);
  }
  return p;
}

// RGB565 word of one endpoint head triple.
__device__ __forceinline__ uint32_t rgb565(float r, float g, float b) {
  return ((uint32_t)quant_bits(r, 31.0f) << 11) | ((uint32_t)quant_bits(g, 63.0f) << 5) | (uint32_t)quant_bits(b, 31.0f);
}

__device__ __forceinline__ Bc1Pal bc1_from_heads(const float* ep, const float* tab = nullptr) {
  return bc1_palette(rgb565(ep[0], ep[1], ep[2]), rgb565(ep[3], ep[4], ep[5]), tab);
}

// 2-bit stored code of the nearest palette entry to colour (r, g, b): first minimum in weight order.
__device__ __forceinline__ uint32_t bc1_code(const Bc1Pal& p, float r, float g, float b) {
  float best = 0.0f;
  uint32_t sh = 0;  // 2 * weight index of the best entry so far
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    const float d0 = __fsub_rn(r, p.pal[n][0]), d1 = __fsub_rn(g, p.pal[n][1]), d2 = __fsub_rn(b, p.pal[n][2]);
    const float e = __fadd_rn(__fadd_rn(__fmul_rn(d0, d0), __fmul_rn(d1, d1)), __fmul_rn(d2, d2));
    if (n == 0) {
      best = e;
    } else {
      sh = e < best ? 2u * n : sh;
      best = e < best ? e : best;
    }
  }
  return (p.map >> sh) & 3u;
}

struct Bc4Pal {
  int e0, e1;
  bool eight;
  uint32_t map;  // stored 3-bit code of weight index n at bits 3n
  float pal[8];  // weight order
};

// Palette of two quantised 8-bit endpoints: eight-value mode when e0 > e1, else six values plus 0 and
// 255.  Stored codes in weight order: eight 0,2,3,4,5,6,7,1; six 6,0,2,3,4,5,1,7.
__device__ __forceinline__ Bc4Pal bc4_palette(int e0, int e1, const float* tab = nullptr) {
  Bc4Pal p;
  p.e0 = e0;
  p.e1 = e1;
  p.eight = e0 > e1;
  int v[8];
  if (p.eight) {
    v[0] = e0;
    v[7] = e1;
#pragma unroll
    for (int j = 1; j <= 6; ++j) v[j] = ((7 - j) * e0 + j * e1 + 3) / 7;
  } else {
    v[0] = 0;
    v[1] = e0;
    v[6] = e1;
    v[7] = 255;
#pragma unroll
    for (int j = 1; j <= 4; ++j) v[1 + j] = ((5 - j) * e0 + j * e1 + 2) / 5;
  }
  constexpr uint32_t kMap8 = 0u | 2u << 3 | 3u << 6 | 4u << 9 | 5u << 12 | 6u << 15 | 7u << 18 | 1u << 21;
  constexpr uint32_t kMap6 = 6u | 0u << 3 | 2u << 6 | 3u << 9 | 4u << 12 | 5u << 15 | 1u << 18 | 7u << 21;
  p.map = p.eight ? kMap8 : kMap6;
#pragma unroll
  for (int n = 0; n < 8; ++n) p.pal[n] = unit8(v[n], tab);
  return p;
}

__device__ __forceinline__ Bc4Pal bc4_from_heads(const float* ep, const float* tab = nullptr) {
  return bc4_palette(quant_bits(ep[0], 255.0f), quant_bits(ep[1], 255.0f), tab);
}

// 3-bit stored code of the nearest palette entry to x, first minimum in weight order.  The palette is
// monotone in weight order in both modes (eight: e0 > interpolants > e1; six: 0 <= e0 <= interpolants
// <= e1 <= 1) and rounding is monotone, so the float32 squared distances are unimodal in the weight
// index: the first minimum is the last index whose distance is strictly below its predecessor's.
__device__ __forceinline__ uint32_t bc4_code(const Bc4Pal& p, float x) {
  float prev;
  {
    const float d = __fsub_rn(x, p.pal[0]);
    prev = __fmul_rn(d, d);
  }
  uint32_t sh = 0;  // 3 * weight index of the first minimum so far
#pragma unroll
  for (int n = 1; n < 8; ++n) {
    const float d = __fsub_rn(x, p.pal[n]);
    const float e = __fmul_rn(d, d);
    sh = e < prev ? 3u * n : sh;
    prev = e;
  }
  return (p.map >> sh) & 7u;
}

// Naive approach (Sec. 3.1): the weight index n of the quantised weight nearest to a predicted weight
// w, |w - w_n| in float32 with the first minimum taken (ties to the smaller n); *wn receives w_n.
// BC1: w_n = n/3; BC4: n/7 in eight-value mode, (n-1)/5 for n = 1..6 in six-value mode (the entries 0
// and 7 are the constants 0 and 1, which carry no weight).  The table values are float32 quotients.
__device__ __forceinline__ int naive_index_bc1(float w, float* wn) {
  constexpr float kW[4] = {0.0f, 1.0f / 3.0f, 2.0f / 3.0f, 1.0f};
  float best = fabsf(__fsub_rn(w, kW[0])), v = kW[0];
  int n_best = 0;
#pragma unroll
  for (int n = 1; n < 4; ++n) {
    const float d = fabsf(__fsub_rn(w, kW[n]));
    const bool take = d < best;
    n_best = take ? n : n_best;
    v = take ? kW[n] : v;
    best = take ? d : best;
  }
  *wn = v;
  return n_best;
}

__device__ __forceinline__ int naive_index_bc4(float w, bool eight, float* wn) {
  constexpr float kW8[8] = {0.0f, 1.0f / 7.0f, 2.0f / 7.0f, 3.0f / 7.0f, 4.0f / 7.0f, 5.0f / 7.0f, 6.0f / 7.0f, 1.0f};
  constexpr float kW6[8] = {0.0f, 1.0f / 5.0f, 2.0f / 5.0f, 3.0f / 5.0f, 4.0f / 5.0f, 1.0f, 0.0f, 0.0f};
  const int count = eight ? 8 : 6, first = eight ? 0 : 1;
  float best = 0.0f, v = 0.0f;
  int n_best = first;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float wk = eight ? kW8[k] : kW6[k];
    const float d = fabsf(__fsub_rn(w, wk));
    const bool take = k == 0 || (k < count && d < best);
    n_best = take ? first + k : n_best;
    v = take ? wk : v;
    best = take ? d : best;
  }
  *wn = v;
  return n_best;
}

}  // namespace dev
}  // namespace ntbc
