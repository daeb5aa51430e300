// BC1 / BC4 on gfx950: the integer reference encoder, the decoder, per-block SSE and the per-block
// fallback.  One thread per 4x4 block; everything is exact integer arithmetic.
//
// Format (paper Sec. 1, Sec. 2.1; Eq. palette and Eq. weightBC4): BC1 = two RGB565 endpoints and
// sixteen 2-bit codes; four colours (c0 > c1: endpoints and the two thirds) or three plus black
// (c0 <= c1: endpoints, midpoint, black).  BC4 = two 8-bit endpoints and sixteen 3-bit codes; eight
// values (e0 > e1: endpoints and six sevenths) or six plus 0 and 255 (e0 <= e1: endpoints, four fifths).
// Endpoints expand to 8 bits by bit replication; interpolants round to the nearest integer (thirds,
// fifths and sevenths of integers never tie; the BC1 midpoint rounds halves up).
//
// Weight ("logical") order n: the order of w_n in Eq. palette / Eq. weightBC4 -- BC1 codes 0,2,3,1;
// BC4 eight-value codes 0,2,3,4,5,6,7,1; BC4 six-value codes 6 (=0),0,2,3,4,5,1,7 (=255).  Ties between
// palette entries go to the smallest n.
//
// The reference encoder (the paper's training targets come from a third-party encoder with two
// refinement steps, Sec. 4.1) is this project's REF-BC1 / REF-BC4 algorithm:
//   BC1: candidate A = farthest texel pair (lexicographically first on ties); candidate B = per-channel
//   bounding box inset by range/16, the diagonal of each channel flipped when its integer covariance
//   with the widest channel is negative; each quantised to the nearest 565 code, put in four-colour
//   order (c0 == c1 -> all codes 0), texels coded by least squared error; the smaller SSE wins (ties A);
//   then two least-squares steps (exact rational endpoints, rounded half up to 5/6 bits), each kept
//   only if the SSE strictly falls.
//   BC4: candidates (max, min) and (min, max) of the texels other than 0/255; two least-squares steps
//   each in its own mode (sevenths, or fifths without the 0/255 texels), dropped if they leave the mode
//   or do not lower the SSE; the smaller SSE wins (ties: the first).
#include <algorithm>

#include "common.h"

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int expand5(int v) { return (v << 3) | (v >> 2); }
__device__ __forceinline__ int expand6(int v) { return (v << 2) | (v >> 4); }

__device__ __forceinline__ void rgb_of_565(uint32_t c, int e[3]) {
  e[0] = expand5((c >> 11) & 31);
  e[1] = expand6((c >> 5) & 63);
  e[2] = expand5(c & 31);
}

// Palette in weight order n = 0..3 (codes 0,2,3,1) for four-colour blocks; for c0 <= c1 the entries are
// code 0, code 2 (midpoint), code 3 (black), code 1.
__device__ __forceinline__ void bc1_palette_logical(uint32_t c0, uint32_t c1, int pal[4][3]) {
  int a[3], b[3];
  rgb_of_565(c0, a);
  rgb_of_565(c1, b);
  const bool four = c0 > c1;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    pal[0][c] = a[c];
    pal[3][c] = b[c];
    pal[1][c] = four ? (2 * a[c] + b[c] + 1) / 3 : (a[c] + b[c] + 1) >> 1;
    pal[2][c] = four ? (a[c] + 2 * b[c] + 1) / 3 : 0;
  }
}

__device__ __forceinline__ uint32_t bc1_code_of(int n) { return (0x78u >> (2 * n)) & 3u; }  // 0,2,3,1

struct Bc1Enc {
  uint32_t c0, c1;
  uint32_t codes;    // 2 bits per texel, stored codes
  uint32_t logical;  // 2 bits per texel, weight order
  int sse;
};

__device__ __forceinline__ uint32_t pack565(const int q[3]) {
  return ((uint32_t)q[0] << 11) | ((uint32_t)q[1] << 5) | (uint32_t)q[2];
}

__device__ Bc1Enc bc1_finish(const int q0[3], const int q1[3], const int p[16][3]) {
  Bc1Enc st;
  uint32_t c0 = pack565(q0), c1 = pack565(q1);
  if (c0 < c1) {
    uint32_t t = c0;
    c0 = c1;
    c1 = t;
  }
  st.c0 = c0;
  st.c1 = c1;
  int pal[4][3];
  bc1_palette_logical(c0, c1, pal);
  st.codes = 0;
  st.logical = 0;
  st.sse = 0;
  if (c0 == c1) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int d0 = p[i][0] - pal[0][0], d1 = p[i][1] - pal[0][1], d2 = p[i][2] - pal[0][2];
      st.sse += d0 * d0 + d1 * d1 + d2 * d2;
    }
    return st;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    int best = 0x7fffffff, bn = 0;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int d0 = p[i][0] - pal[n][0], d1 = p[i][1] - pal[n][1], d2 = p[i][2] - pal[n][2];
      const int e = d0 * d0 + d1 * d1 + d2 * d2;
      if (e < best) {
        best = e;
        bn = n;
      }
    }
    st.sse += best;
    st.logical |= (uint32_t)bn << (2 * i);
    st.codes |= bc1_code_of(bn) << (2 * i);
  }
  return st;
}

__device__ __forceinline__ int quant5(int v) { return (v * 31 + 127) / 255; }
__device__ __forceinline__ int quant6(int v) { return (v * 63 + 127) / 255; }

// round-half-up of (num/den) * mul / 255 with num clamped to [0, 255 den], den > 0
__device__ __forceinline__ int ratio_code(long long num, long long den, int mul) {
  num = num < 0 ? 0 : (num > 255 * den ? 255 * den : num);
  return (int)((2 * num * mul + 255 * den) / (2 * 255 * den));
}

__device__ void bc1_refine(Bc1Enc& st, const int p[16][3]) {
  long long saa = 0, sbb = 0, sab = 0, sap[3] = {0, 0, 0}, sbp[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int n = (st.logical >> (2 * i)) & 3;
    const int a = 3 - n, b = n;
    saa += a * a;
    sbb += b * b;
    sab += a * b;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sap[c] += a * p[i][c];
      sbp[c] += b * p[i][c];
    }
  }
  const long long det = saa * sbb - sab * sab;
  if (det <= 0) return;
  int qa[3], qb[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int mul = c == 1 ? 63 : 31;
    qa[c] = ratio_code(3 * (sbb * sap[c] - sab * sbp[c]), det, mul);
    qb[c] = ratio_code(3 * (saa * sbp[c] - sab * sap[c]), det, mul);
  }
  const Bc1Enc nw = bc1_finish(qa, qb, p);
  if (nw.sse < st.sse) st = nw;
}

// Optimal single-colour endpoints (step 8 of REF-BC1): for every value v, the code pair (a, b) of 5-bit
// (g_single5) or 6-bit (g_single6) endpoints whose four-colour 2/3 point (2 E(a) + E(b) + 1) / 3 is
// nearest to v, ties to the smallest a, then the smallest b; entry = a | b << 8.  Filled on the device
// by k_single_colour_init before each encode (the same values every time): one workgroup per (value,
// table), its threads taking every 256th candidate pair and the minimum of (error, a, b) reduced in
// that order.
__device__ uint16_t g_single5[256];
__device__ uint16_t g_single6[256];

__global__ void __launch_bounds__(256) k_single_colour_init() {
  __shared__ unsigned best_s[4];
  const int v = blockIdx.x;
  const int bits = blockIdx.y == 0 ? 5 : 6;
  const int n = 1 << bits;
  unsigned best = 0xFFFFFFFFu;  // error << 16 | a << 8 | b: the smallest error, then a, then b
  for (int k = threadIdx.x; k < n * n; k += 256) {
    const int a = k / n, b = k % n;
    const int ea = bits == 5 ? expand5(a) : expand6(a), eb = bits == 5 ? expand5(b) : expand6(b);
    const unsigned key = ((unsigned)abs((2 * ea + eb + 1) / 3 - v) << 16) | ((unsigned)a << 8) | (unsigned)b;
    best = key < best ? key : best;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned o = (unsigned)__shfl_xor((int)best, off);
    best = o < best ? o : best;
  }
  if ((threadIdx.x & 63) == 0) best_s[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) best = best_s[w] < best ? best_s[w] : best;
    (bits == 5 ? g_single5 : g_single6)[v] = (uint16_t)(((best >> 8) & 255u) | ((best & 255u) << 8));
  }
}

__device__ Bc1Enc bc1_encode_block(const int p[16][3]) {
  // candidate A: farthest pair
  int best = -1, bi = 0, bj = 1;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
#pragma unroll
    for (int j = i + 1; j < 16; ++j) {
      const int d0 = p[i][0] - p[j][0], d1 = p[i][1] - p[j][1], d2 = p[i][2] - p[j][2];
      const int d = d0 * d0 + d1 * d1 + d2 * d2;
      if (d > best) {
        best = d;
        bi = i;
        bj = j;
      }
    }
  }
  int qa0[3] = {quant5(p[bi][0]), quant6(p[bi][1]), quant5(p[bi][2])};
  int qa1[3] = {quant5(p[bj][0]), quant6(p[bj][1]), quant5(p[bj][2])};
  Bc1Enc st = bc1_finish(qa0, qa1, p);
  // candidate B: inset bounding box, diagonal signed by covariance with the widest channel
  int mn[3] = {255, 255, 255}, mx[3] = {0, 0, 0}, sum[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < 16; ++i) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      mn[c] = min(mn[c], p[i][c]);
      mx[c] = max(mx[c], p[i][c]);
      sum[c] += p[i][c];
    }
  }
  int m = 0;
  if (mx[1] - mn[1] > mx[m] - mn[m]) m = 1;
  if (mx[2] - mn[2] > mx[m] - mn[m]) m = 2;
  int b0[3], b1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int inset = (mx[c] - mn[c]) >> 4;
    const int lo = mn[c] + inset, hi = mx[c] - inset;
    int cross = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) cross += p[i][c] * p[i][m];
    const int cov = 16 * cross - sum[c] * sum[m];
    b0[c] = cov < 0 ? lo : hi;
    b1[c] = cov < 0 ? hi : lo;
  }
  int qb0[3] = {quant5(b0[0]), quant6(b0[1]), quant5(b0[2])};
  int qb1[3] = {quant5(b1[0]), quant6(b1[1]), quant5(b1[2])};
  const Bc1Enc stb = bc1_finish(qb0, qb1, p);
  if (stb.sse < st.sse) st = stb;
  bc1_refine(st, p);
  bc1_refine(st, p);
  // step 8: a one-colour block also tries the optimal single-colour endpoints
  bool uniform = true;
#pragma unroll
  for (int i = 1; i < 16; ++i) uniform &= p[i][0] == p[0][0] && p[i][1] == p[0][1] && p[i][2] == p[0][2];
  if (uniform) {
    const uint32_t r = g_single5[p[0][0]], g = g_single6[p[0][1]], b = g_single5[p[0][2]];
    const int q0[3] = {(int)(r & 255u), (int)(g & 255u), (int)(b & 255u)};
    const int q1[3] = {(int)(r >> 8), (int)(g >> 8), (int)(b >> 8)};
    const Bc1Enc sc = bc1_finish(q0, q1, p);
    if (sc.sse < st.sse) st = sc;
  }
  return st;
}

// ---------------------------------------------------------------------------------------------- BC4
__device__ __forceinline__ void bc4_palette_logical(int e0, int e1, int pal[8]) {
  if (e0 > e1) {
    pal[0] = e0;
    pal[7] = e1;
#pragma unroll
    for (int j = 1; j <= 6; ++j) pal[j] = ((7 - j) * e0 + j * e1 + 3) / 7;
  } else {
    pal[0] = 0;
    pal[1] = e0;
    pal[6] = e1;
    pal[7] = 255;
#pragma unroll
    for (int j = 1; j <= 4; ++j) pal[1 + j] = ((5 - j) * e0 + j * e1 + 2) / 5;
  }
}

__device__ __forceinline__ uint32_t bc4_code_of(int n, bool eight) {
  // eight-value: 0,2,3,4,5,6,7,1   six-value: 6,0,2,3,4,5,1,7
  if (eight) return n == 0 ? 0u : (n == 7 ? 1u : (uint32_t)(n + 1));
  return n == 0 ? 6u : (n == 1 ? 0u : (n == 6 ? 1u : (n == 7 ? 7u : (uint32_t)n)));
}

struct Bc4Enc {
  int e0, e1;
  uint64_t codes;    // 3 bits per texel
  uint64_t logical;  // 3 bits per texel
  int sse;
};

__device__ Bc4Enc bc4_finish(int e0, int e1, const int v[16]) {
  Bc4Enc st;
  st.e0 = e0;
  st.e1 = e1;
  st.codes = 0;
  st.logical = 0;
  st.sse = 0;
  int pal[8];
  bc4_palette_logical(e0, e1, pal);
  const bool eight = e0 > e1;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    int best = 0x7fffffff, bn = 0;
#pragma unroll
    for (int n = 0; n < 8; ++n) {
      const int d = v[i] - pal[n];
      if (d * d < best) {
        best = d * d;
        bn = n;
      }
    }
    st.sse += best;
    st.logical |= (uint64_t)bn << (3 * i);
    st.codes |= (uint64_t)bc4_code_of(bn, eight) << (3 * i);
  }
  return st;
}

__device__ void bc4_refine(Bc4Enc& st, const int v[16]) {
  const bool eight = st.e0 > st.e1;
  long long saa = 0, sbb = 0, sab = 0, sav = 0, sbv = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int n = (int)((st.logical >> (3 * i)) & 7);
    const bool inc = eight || (n >= 1 && n <= 6);
    const int a = inc ? (eight ? 7 - n : 6 - n) : 0;
    const int b = inc ? (eight ? n : n - 1) : 0;
    saa += a * a;
    sbb += b * b;
    sab += a * b;
    sav += a * v[i];
    sbv += b * v[i];
  }
  const long long det = saa * sbb - sab * sab;
  if (det <= 0) return;
  const long long scale = eight ? 7 : 5;
  long long na = scale * (sbb * sav - sab * sbv);
  long long nb = scale * (saa * sbv - sab * sav);
  na = na < 0 ? 0 : (na > 255 * det ? 255 * det : na);
  nb = nb < 0 ? 0 : (nb > 255 * det ? 255 * det : nb);
  const int ea = (int)((2 * na + det) / (2 * det));
  const int eb = (int)((2 * nb + det) / (2 * det));
  if (eight ? !(ea > eb) : !(ea <= eb)) return;
  const Bc4Enc nw = bc4_finish(ea, eb, v);
  if (nw.sse < st.sse) st = nw;
}

__device__ Bc4Enc bc4_encode_block(const int v[16]) {
  int mn = 255, mx = 0, imn = 256, imx = -1;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    mn = min(mn, v[i]);
    mx = max(mx, v[i]);
    if (v[i] > 0 && v[i] < 255) {
      imn = min(imn, v[i]);
      imx = max(imx, v[i]);
    }
  }
  Bc4Enc s8 = bc4_finish(mx, mn, v);
  bc4_refine(s8, v);
  bc4_refine(s8, v);
  const bool has = imx >= 0;
  Bc4Enc s6 = bc4_finish(has ? imn : 0, has ? imx : 0, v);
  bc4_refine(s6, v);
  bc4_refine(s6, v);
  return s6.sse < s8.sse ? s6 : s8;
}

// ------------------------------------------------------------------------------------------ kernels
__global__ void __launch_bounds__(kThreads) k_encode_ref_bc1(const uint8_t* __restrict__ tex, int bw, int bh,
                                                       int pitch, uint64_t* __restrict__ out,
                                                       int32_t* __restrict__ sse_out) {
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (b >= (int64_t)bw * bh) return;
  const int bx = (int)(b % bw), by = (int)(b / bw);
  int p[16][3];
#pragma unroll
  for (int y = 0; y < 4; ++y) {
    const uint8_t* row = tex + (int64_t)(4 * by + y) * pitch + (int64_t)12 * bx;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
#pragma unroll
      for (int c = 0; c < 3; ++c) p[4 * y + x][c] = row[3 * x + c];
    }
  }
  const Bc1Enc st = bc1_encode_block(p);
  out[b] = (uint64_t)st.c0 | ((uint64_t)st.c1 << 16) | ((uint64_t)st.codes << 32);
  if (sse_out) sse_out[b] = st.sse;
}

__global__ void __launch_bounds__(kThreads) k_encode_ref_bc4(const uint8_t* __restrict__ tex, int bw, int bh,
                                                       int pitch, uint64_t* __restrict__ out,
                                                       int32_t* __restrict__ sse_out) {
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (b >= (int64_t)bw * bh) return;
  const int bx = (int)(b % bw), by = (int)(b / bw);
  int v[16];
#pragma unroll
  for (int y = 0; y < 4; ++y) {
    const uint8_t* row = tex + (int64_t)(4 * by + y) * pitch + (int64_t)4 * bx;
#pragma unroll
    for (int x = 0; x < 4; ++x) v[4 * y + x] = row[x];
  }
  const Bc4Enc st = bc4_encode_block(v);
  out[b] = (uint64_t)st.e0 | ((uint64_t)st.e1 << 8) | (st.codes << 16);
  if (sse_out) sse_out[b] = st.sse;
}

// Decoded palettes indexed by the stored code.
__device__ __forceinline__ void bc1_palette_by_code(uint32_t c0, uint32_t c1, int pal[4][3]) {
  int l[4][3];
  bc1_palette_logical(c0, c1, l);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    pal[0][c] = l[0][c];
    pal[1][c] = l[3][c];
    pal[2][c] = l[1][c];
    pal[3][c] = l[2][c];
  }
}

__device__ __forceinline__ void bc4_palette_by_code(int e0, int e1, int pal[8]) {
  pal[0] = e0;
  pal[1] = e1;
  if (e0 > e1) {
#pragma unroll
    for (int j = 1; j <= 6; ++j) pal[1 + j] = ((7 - j) * e0 + j * e1 + 3) / 7;
  } else {
#pragma unroll
    for (int j = 1; j <= 4; ++j) pal[1 + j] = ((5 - j) * e0 + j * e1 + 2) / 5;
    pal[6] = 0;
    pal[7] = 255;
  }
}

__global__ void __launch_bounds__(kThreads) k_decode_bc1(const uint64_t* __restrict__ blocks, int bw, int bh,
                                                   uint8_t* __restrict__ tex, int pitch) {
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (b >= (int64_t)bw * bh) return;
  const int bx = (int)(b % bw), by = (int)(b / bw);
  const uint64_t w = blocks[b];
  int pal[4][3];
  bc1_palette_by_code((uint32_t)(w & 0xFFFF), (uint32_t)((w >> 16) & 0xFFFF), pal);
  const uint32_t idx = (uint32_t)(w >> 32);
#pragma unroll
  for (int y = 0; y < 4; ++y) {
    uint8_t* row = tex + (int64_t)(4 * by + y) * pitch + (int64_t)12 * bx;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int code = (idx >> (2 * (4 * y + x))) & 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) row[3 * x + c] = (uint8_t)pal[code][c];
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_decode_bc4(const uint64_t* __restrict__ blocks, int bw, int bh,
                                                   uint8_t* __restrict__ tex, int pitch) {
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (b >= (int64_t)bw * bh) return;
  const int bx = (int)(b % bw), by = (int)(b / bw);
  const uint64_t w = blocks[b];
  int pal[8];
  bc4_palette_by_code((int)(w & 0xFF), (int)((w >> 8) & 0xFF), pal);
  const uint64_t idx = w >> 16;
#pragma unroll
  for (int y = 0; y < 4; ++y) {
    uint32_t packed = 0;
#pragma unroll
    for (int x = 0; x < 4; ++x) packed |= (uint32_t)pal[(idx >> (3 * (4 * y + x))) & 7] << (8 * x);
    uint8_t* row = tex + (int64_t)(4 * by + y) * pitch + (int64_t)4 * bx;
    if ((((uintptr_t)row) & 3) == 0) {
      *reinterpret_cast<uint32_t*>(row) = packed;
    } else {
#pragma unroll
      for (int x = 0; x < 4; ++x) row[x] = (uint8_t)(packed >> (8 * x));
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_block_sse(const uint64_t* __restrict__ blocks,
                                                  const uint8_t* __restrict__ tex, int bw, int bh,
                                                  int pitch, int fmt, int32_t* __restrict__ sse) {
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (b >= (int64_t)bw * bh) return;
  const int bx = (int)(b % bw), by = (int)(b / bw);
  const uint64_t w = blocks[b];
  int total = 0;
  if (fmt == NTBC_BC1) {
    int pal[4][3];
    bc1_palette_by_code((uint32_t)(w & 0xFFFF), (uint32_t)((w >> 16) & 0xFFFF), pal);
    const uint32_t idx = (uint32_t)(w >> 32);
    for (int y = 0; y < 4; ++y) {
      const uint8_t* row = tex + (int64_t)(4 * by + y) * pitch + (int64_t)12 * bx;
      for (int x = 0; x < 4; ++x) {
        const int code = (idx >> (2 * (4 * y + x))) & 3;
        for (int c = 0; c < 3; ++c) {
          const int d = (int)row[3 * x + c] - pal[code][c];
          total += d * d;
        }
      }
    }
  } else {
    int pal[8];
    bc4_palette_by_code((int)(w & 0xFF), (int)((w >> 8) & 0xFF), pal);
    const uint64_t idx = w >> 16;
    for (int y = 0; y < 4; ++y) {
      const uint8_t* row = tex + (int64_t)(4 * by + y) * pitch + (int64_t)4 * bx;
      for (int x = 0; x < 4; ++x) {
        const int d = (int)row[x] - pal[(idx >> (3 * (4 * y + x))) & 7];
        total += d * d;
      }
    }
  }
  sse[b] = total;
}

__global__ void __launch_bounds__(kThreads) k_fallback(const uint64_t* __restrict__ ntbc_words,
                                                 const uint64_t* __restrict__ ref_words,
                                                 const int32_t* __restrict__ sse_n,
                                                 const int32_t* __restrict__ sse_r, int64_t n, float kappa,
                                                 float delta, uint64_t* __restrict__ out,
                                                 int32_t* __restrict__ count) {
  // grid-stride over the blocks; the replaced count is summed per wavefront (ballot), then per
  // workgroup in LDS, and added with one atomic per workgroup (same-address atomics serialise)
  __shared__ int part[kThreads / 64];
  int mine = 0;
  for (int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x; b - threadIdx.x < n; b += (int64_t)gridDim.x * kThreads) {
    bool replaced = false;
    if (b < n) {
      const float limit = kappa * (float)sse_r[b] + delta;
      replaced = (float)sse_n[b] > limit;
      out[b] = replaced ? ref_words[b] : ntbc_words[b];
    }
    mine += (int)__popcll(__ballot(replaced));
  }
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < kThreads / 64; ++w) tot += part[w];
    if (tot != 0) atomicAdd(count, tot);
  }
}

int check_texture(const void* tex, int32_t width, int32_t height, int32_t pitch, int32_t format) {
  NTBC_REQUIRE(tex != nullptr, "texture pointer is NULL");
  NTBC_REQUIRE(format == NTBC_BC1 || format == NTBC_BC4, "format %d is not NTBC_BC1 or NTBC_BC4", format);
  NTBC_REQUIRE(width > 0 && height > 0 && width % 4 == 0 && height % 4 == 0,
               "texture %dx%d must be positive multiples of 4", width, height);
  const int ch = format == NTBC_BC1 ? 3 : 1;
  NTBC_REQUIRE(pitch >= width * ch, "row_pitch %d smaller than width*channels %d", pitch, width * ch);
  return NTBC_OK;
}

}  // namespace

extern "C" int ntbc_bc_encode_ref(const uint8_t* texels, int32_t width, int32_t height, int32_t row_pitch,
                                  int32_t format, uint64_t* blocks_out, int32_t* sse_out, void* stream) {
  int st = check_texture(texels, width, height, row_pitch, format);
  if (st != NTBC_OK) return st;
  NTBC_REQUIRE(blocks_out != nullptr, "blocks_out is NULL");
  const int bw = width / 4, bh = height / 4;
  const int64_t n = (int64_t)bw * bh;
  const dim3 grid((unsigned)ntbc::ceil_div(n, kThreads));
  if (format == NTBC_BC1) {
    hipLaunchKernelGGL(k_single_colour_init, dim3(256, 2), dim3(256), 0, ntbc::as_stream(stream));
    hipLaunchKernelGGL(k_encode_ref_bc1, grid, dim3(kThreads), 0, ntbc::as_stream(stream), texels, bw, bh,
                       row_pitch, blocks_out, sse_out);
  }
  else
    hipLaunchKernelGGL(k_encode_ref_bc4, grid, dim3(kThreads), 0, ntbc::as_stream(stream), texels, bw, bh,
                       row_pitch, blocks_out, sse_out);
  return ntbc::check_launch("ntbc_bc_encode_ref");
}

// One thread per (block, texel row): the row's 4 texels (4 * ch bytes) to their place in the block-major copy.
__global__ void __launch_bounds__(kThreads) k_texels_to_blocks(const uint8_t* __restrict__ tex, int bw, int bh, int pitch,
                                                               int ch, uint8_t* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= (int64_t)bw * bh * 4) return;
  const int64_t b = e >> 2;
  const int y = (int)(e & 3);
  const int bx = (int)(b % bw), by = (int)(b / bw);
  const uint8_t* src = tex + (int64_t)(4 * by + y) * pitch + (int64_t)(4 * bx) * ch;
  uint8_t* dst = out + (b * 16 + 4 * y) * ch;
  for (int k = 0; k < 4 * ch; ++k) dst[k] = src[k];
}

extern "C" int ntbc_texels_to_blocks(const uint8_t* texels, int32_t width, int32_t height, int32_t row_pitch,
                                     int32_t format, uint8_t* blocks_out, void* stream) {
  int st = check_texture(texels, width, height, row_pitch, format);
  if (st != NTBC_OK) return st;
  NTBC_REQUIRE(blocks_out != nullptr, "blocks_out is NULL");
  const int bw = width / 4, bh = height / 4;
  const int64_t n = (int64_t)bw * bh * 4;
  if (n == 0) return NTBC_OK;
  hipLaunchKernelGGL(k_texels_to_blocks, dim3((unsigned)ntbc::ceil_div(n, kThreads)), dim3(kThreads), 0,
                     ntbc::as_stream(stream), texels, bw, bh, row_pitch, format == NTBC_BC1 ? 3 : 1, blocks_out);
  return ntbc::check_launch("ntbc_texels_to_blocks");
}

extern "C" int ntbc_bc_decode(const uint64_t* blocks, int32_t width, int32_t height, int32_t format,
                              uint8_t* texels_out, int32_t row_pitch, void* stream) {
  int st = check_texture(texels_out, width, height, row_pitch, format);
  if (st != NTBC_OK) return st;
  NTBC_REQUIRE(blocks != nullptr, "blocks is NULL");
  const int bw = width / 4, bh = height / 4;
  const int64_t n = (int64_t)bw * bh;
  const dim3 grid((unsigned)ntbc::ceil_div(n, kThreads));
  if (format == NTBC_BC1)
    hipLaunchKernelGGL(k_decode_bc1, grid, dim3(kThreads), 0, ntbc::as_stream(stream), blocks, bw, bh,
                       texels_out, row_pitch);
  else
    hipLaunchKernelGGL(k_decode_bc4, grid, dim3(kThreads), 0, ntbc::as_stream(stream), blocks, bw, bh,
                       texels_out, row_pitch);
  return ntbc::check_launch("ntbc_bc_decode");
}

extern "C" int ntbc_block_sse(const uint64_t* blocks, const uint8_t* texels, int32_t width, int32_t height,
                              int32_t row_pitch, int32_t format, int32_t* sse_out, void* stream) {
  int st = check_texture(texels, width, height, row_pitch, format);
  if (st != NTBC_OK) return st;
  NTBC_REQUIRE(blocks != nullptr && sse_out != nullptr, "blocks or sse_out is NULL");
  const int bw = width / 4, bh = height / 4;
  const int64_t n = (int64_t)bw * bh;
  hipLaunchKernelGGL(k_block_sse, dim3((unsigned)ntbc::ceil_div(n, kThreads)), dim3(kThreads), 0,
                     ntbc::as_stream(stream), blocks, texels, bw, bh, row_pitch, format, sse_out);
  return ntbc::check_launch("ntbc_block_sse");
}

extern "C" int ntbc_fallback(const uint64_t* ntbc_words, const uint64_t* ref, const int32_t* sse_ntbc,
                             const int32_t* sse_ref, int64_t n_blocks, float kappa, float delta, uint64_t* out,
                             int32_t* n_fallback, void* stream) {
  NTBC_REQUIRE(ntbc_words && ref && sse_ntbc && sse_ref && out && n_fallback, "NULL pointer argument");
  NTBC_REQUIRE(n_blocks >= 0, "n_blocks %lld < 0", (long long)n_blocks);
  if (n_blocks == 0) return NTBC_OK;
  hipLaunchKernelGGL(k_fallback, dim3((unsigned)std::min<int64_t>(ntbc::ceil_div(n_blocks, kThreads), 1024)), dim3(kThreads), 0,
                     ntbc::as_stream(stream), ntbc_words, ref, sse_ntbc, sse_ref, n_blocks, kappa, delta, out,
                     n_fallback);
  return ntbc::check_launch("ntbc_fallback");
}
