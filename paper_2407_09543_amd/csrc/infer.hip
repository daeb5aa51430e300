// NTBC inference on gfx950 (paper Sec. 3.2, Fig. NTBC inference): block coordinate -> bilinear grid
// features -> MLP -> sigmoid heads -> quantised endpoints, nearest-palette indices, packed BC words,
// fused into one kernel per precision.
//
// Layout of the MLP on the matrix cores.  Block positions are the N (column) dimension of every
// product, neurons the M (row) dimension: D[neuron][position] = W[neuron][k] * H[k][position].  A wave
// owns P positions for the whole network; its activations never leave registers: the accumulator
// layout of one layer's output tile is reused directly as the B operand of the next layer, and the
// next layer's weight columns are permuted on the host side of the kernel (k_pack_weights) to match.
//
//   BF16 / FP16 (v_mfma_f32_32x32x16_{bf16,f16}, P = 32): lane l holds position j = l%32 and row
//     group g = l/32;
//     accumulator v of output tile t is neuron 32t + 8(v/4) + 4g + v%4.  Values v = 8h..8h+7 of tile
//     t become the eight B-operand values of K-step s = 2t+h; so K-step s, lane group g, element m
//     of a hidden layer's input is neuron 32(s/2) + 16(s%2) + 8(m/4) + 4g + m%4.  The first layer's
//     input (grid features) uses the identity order c = 16s + 8g + m.
//   FP32 (v_mfma_f32_16x16x4f32, P = 16): lane l holds position j = l%16 and row group g = l/16;
//     accumulator v of tile t is neuron 16t + 4g + v and becomes K-step s = 4t+v: K-step s, group g
//     of a hidden layer's input is neuron 16(s/4) + 4g + s%4; first layer c = 4s + g.
//
// Weights (A operands) are read from the packed copy in the workspace, each lane's operand being one
// contiguous 16-byte (16-bit formats) or 4-byte (FP32) load; the copy is made by k_pack_lp / k_pack_f32
// unless the caller says it is current.
#include <algorithm>
#include <mutex>
#include <vector>

#include "common.h"
#include "device.h"

// The build compiles this file once per part so that the many kernel instances compile in parallel:
// NTBC_INFER_PART = 0 holds the host code, the FP32 kernels and the weight packing, 1-3 the
// single-range 16-bit/FP8 instances (BF16, FP16, FP8), 4-6 the batched ones (BF16 with 4-wave tiles,
// FP16, FP8), 7-8 the BF16 batched ones with 2- and 8-wave tiles, 9 the paper-layout model.  Without
// the macro one translation unit holds everything.
#ifndef NTBC_INFER_PART
#define NTBC_INFER_PART -1
#endif
#define NTBC_PART(k) (NTBC_INFER_PART < 0 || NTBC_INFER_PART == (k))

namespace {

using namespace ntbc;

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef short i16x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u32x4 mk4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) { return u32x4{a, b, c, d}; }

// The reduced-precision matrix formats: bfloat16 (8 significant bits, float32's range), IEEE half (11
// significant bits, the precision the paper evaluates its networks in) and FP8 E4M3 (OCP, 4
// significant bits, largest finite 448) with per-layer power-of-two scales.  All use a 32x32x16
// matrix-core shape with float32 accumulation and the same operand layouts (lane l: row/column l%32,
// K elements 8(l/32) .. 8(l/32)+7); an operand is eight values: 16 bytes, or 8 bytes for FP8.
enum class Lp { BF16, FP16, FP8 };

template <Lp L> struct LpOp { typedef u32x4 type; };
template <> struct LpOp<Lp::FP8> { typedef u32x2 type; };

// Two floats -> two 16-bit values (round to nearest even) in one 32-bit word (v_cvt_pk_*_f32).
template <Lp L>
__device__ __forceinline__ uint32_t cvt2(float lo, float hi) {
  if constexpr (L == Lp::BF16)
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{lo, hi}, bf16x2_t));
  else
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{lo, hi}, f16x2_t));
}

// Four floats -> four E4M3 bytes (round to nearest even), saturating at +-448 like the E4M3FN
// conversion of the oracle (the hardware conversion would give NaN beyond the range).
__device__ __forceinline__ float sat448(float x) { return fminf(fmaxf(x, -448.0f), 448.0f); }
__device__ __forceinline__ uint32_t cvt4_fp8(float a, float b, float c, float d) {
  const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(a), sat448(b), 0, false);
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(sat448(c), sat448(d), lo, true);
}

// Eight floats (already divided by the FP8 scale) -> one operand.
template <Lp L>
__device__ __forceinline__ typename LpOp<L>::type x8_of(const float* v) {
  if constexpr (L == Lp::FP8)
    return u32x2{cvt4_fp8(v[0], v[1], v[2], v[3]), cvt4_fp8(v[4], v[5], v[6], v[7])};
  else
    return mk4(cvt2<L>(v[0], v[1]), cvt2<L>(v[2], v[3]), cvt2<L>(v[4], v[5]), cvt2<L>(v[6], v[7]));
}

template <Lp L>
__device__ __forceinline__ f32x16_t mfma16(const typename LpOp<L>::type& a, const typename LpOp<L>::type& b,
                                           const f32x16_t& c) {
  if constexpr (L == Lp::BF16)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                   0, 0, 0);
  else if constexpr (L == Lp::FP16)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, a), __builtin_bit_cast(f16x8_t, b), c,
                                                  0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(__builtin_bit_cast(long, a), __builtin_bit_cast(long, b), c, 0, 0,
                                                      0);
}

// ReLU of two 16-bit floats in one word: max as signed 16-bit integers against 0 (a negative
// bfloat16 or half has its sign bit set, so it is a negative int16).
__device__ __forceinline__ uint32_t relu16x2(uint32_t x) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(i16x2_t, x), i16x2_t{0, 0}));
}

constexpr int kMaxLayers = 5;
constexpr int kHeadRows = 192;  // head rows of the fused 16-bit/FP8 kernels (six 32-row tiles)
constexpr int kWaves = 2;  // waves per workgroup

struct PackArgs {
  const float* w;           // canonical FP32 weights
  int n_layers;
  int in_dim[kMaxLayers], out_dim[kMaxLayers];
  int64_t w_off[kMaxLayers], b_off[kMaxLayers];
  int ksteps[kMaxLayers], otiles[kMaxLayers];
  int64_t pack_off[kMaxLayers];  // in operand units (16 bytes for 16-bit formats, float for FP32)
  int64_t bias_off[kMaxLayers];  // floats
  int pos_hidden;                // hidden layers use the chained input permutation
  const float* fp8_scales;       // FP8: [n_layers][2] = (s_x, s_w)
  int head_perm;                 // head rows permuted for the register-resident BC epilogue
  int16_t head_src[kHeadRows];   // head_perm: canonical head neuron of packed row r, -1 = zero row
};

struct InferArgs {
  dev::GridView grid;
  const void* wpack;            // packed A operands
  const float* bias;            // padded biases
  int64_t pack_off[kMaxLayers];
  int64_t bias_off[kMaxLayers];
  int ksteps[kMaxLayers], otiles[kMaxLayers];
  int n_layers;
  int head_dim, head_stride;
  int n_textures, formats[NTBC_MAX_TEXTURES], ep_off[NTBC_MAX_TEXTURES], ch_off[NTBC_MAX_TEXTURES];
  int endpoint_dim, channels;
  int naive;                    // weight head (Sec. 3.1): texel i's weight of texture t at endpoint_dim + i*n_textures + t
  int64_t first, n;
  uint64_t* out;                // [n_textures][n]
  float* heads;                 // optional [n][head_dim]
  const float* fp8_scales;      // FP8: [n_layers][2] = (s_x, s_w)
  int64_t stride;               // calibration: block id of sample i is i * stride
  unsigned* amax;               // calibration: per layer, max |layer input| as float bits
  // register-resident BC epilogue: texture k of the slot layout (BC1 textures first, then BC4) is
  // canonical texture reg_tex[k]; reg_ep / reg_ch are its endpoint and colour-channel offsets
  int reg_tex[NTBC_MAX_TEXTURES], reg_ep[NTBC_MAX_TEXTURES], reg_ch[NTBC_MAX_TEXTURES];
};

// ------------------------------------------------------------------------------ weight packing
// 16-bit formats: element (tile t, step s, lane l, m) = W[32t + l%32][col(s, l/32, m)].
__device__ __forceinline__ int bf16_col(int layer, int s, int g, int m) {
  if (layer == 0) return 16 * s + 8 * g + m;
  return 32 * (s / 2) + 16 * (s % 2) + 8 * (m / 4) + 4 * g + (m % 4);
}

__device__ __forceinline__ int f32_col(int layer, int s, int g) {
  if (layer == 0) return 4 * s + g;
  return 16 * (s / 4) + 4 * g + (s % 4);
}

template <Lp L>
__global__ void k_pack_lp(PackArgs a, typename LpOp<L>::type* __restrict__ pack, float* __restrict__ bias) {
  const int layer = blockIdx.y;
  if (layer >= a.n_layers) return;
  // FP8 mode: the middle layers as E4M3 of W * (1/s_w) in float32 (exact for the power-of-two scales);
  // the first layer and the head as bfloat16 operands, each filling two 8-byte units
  const bool wide = L == Lp::FP8 && (layer == 0 || layer == a.n_layers - 1);
  const float inv_w = L == Lp::FP8 && !wide ? 1.0f / a.fp8_scales[2 * layer + 1] : 1.0f;
  const int64_t total = (int64_t)a.otiles[layer] * a.ksteps[layer] * 64;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(e % 64);
    const int s = (int)((e / 64) % a.ksteps[layer]);
    const int t = (int)(e / (64 * (int64_t)a.ksteps[layer]));
    const int prow = 32 * t + (l % 32);
    const int row = a.head_perm && layer == a.n_layers - 1 ? (prow < kHeadRows ? a.head_src[prow] : -1) : prow;
    float v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int col = bf16_col(layer, s, l / 32, m);
      v[m] = (row >= 0 && row < a.out_dim[layer] && col < a.in_dim[layer])
                 ? a.w[a.w_off[layer] + (int64_t)row * a.in_dim[layer] + col]
                 : 0.0f;
    }
    if constexpr (L == Lp::FP8) {
      if (wide) {
        const u32x4 w16 = x8_of<Lp::BF16>(v);
        pack[a.pack_off[layer] + 2 * e] = u32x2{w16[0], w16[1]};
        pack[a.pack_off[layer] + 2 * e + 1] = u32x2{w16[2], w16[3]};
        continue;
      }
#pragma unroll
      for (int m = 0; m < 8; ++m) v[m] *= inv_w;
    }
    pack[a.pack_off[layer] + e] = x8_of<L>(v);
  }
  const int nb = a.otiles[layer] * 32;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x) {
    const int row = a.head_perm && layer == a.n_layers - 1 ? (i < kHeadRows ? a.head_src[i] : -1) : i;
    bias[a.bias_off[layer] + i] = row >= 0 && row < a.out_dim[layer] ? a.w[a.b_off[layer] + row] : 0.0f;
  }
}

__global__ void k_pack_f32(PackArgs a, float* __restrict__ pack, float* __restrict__ bias) {
  const int layer = blockIdx.y;
  if (layer >= a.n_layers) return;
  const int64_t total = (int64_t)a.otiles[layer] * a.ksteps[layer] * 64;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(e % 64);
    const int s = (int)((e / 64) % a.ksteps[layer]);
    const int t = (int)(e / (64 * (int64_t)a.ksteps[layer]));
    const int row = 16 * t + (l % 16);
    const int col = f32_col(layer, s, l / 16);
    pack[a.pack_off[layer] + e] = (row < a.out_dim[layer] && col < a.in_dim[layer])
                                      ? a.w[a.w_off[layer] + (int64_t)row * a.in_dim[layer] + col]
                                      : 0.0f;
  }
  const int nb = a.otiles[layer] * 16;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x)
    bias[a.bias_off[layer] + i] = i < a.out_dim[layer] ? a.w[a.b_off[layer] + i] : 0.0f;
}

// ------------------------------------------------------------------------------ common epilogue
// XCD-aware order: consecutive workgroup ids are dispatched round-robin over the 8 XCDs; give each
// XCD a contiguous run of position tiles so its L2 holds one band of the fine grid levels.
__device__ __forceinline__ int64_t xcd_tile(int64_t wg, int64_t nwg) {
  const int64_t per = nwg / 8, extra = nwg % 8;
  const int64_t x = wg % 8, k = wg / 8;
  return x * per + (x < extra ? x : extra) + k;
}

__device__ __forceinline__ float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

// Sigmoid with the hardware exp2 and reciprocal (each within ~1 ulp): |error| < 3e-7 for |z| < 64.
__device__ __forceinline__ float sigmoid_fast(float z) {
  const float e = __builtin_amdgcn_exp2f(-z * 1.4426950408889634f);
  return __builtin_amdgcn_rcpf(1.0f + e);
}

// Packs the blocks of the wave's P positions from the sigmoid heads in LDS (y: [P][head_stride]).
// Lane layout: position j = lane % P, texel group q = lane / P handles texels q*TPL .. q*TPL+TPL-1.
template <int P>
__device__ void pack_blocks(const InferArgs& a, const float* __restrict__ y, int lane, int64_t pos0,
                            const float* tab = nullptr) {
  constexpr int LPP = 64 / P;   // lanes per position
  constexpr int TPL = 16 / LPP; // texels per lane
  const int j = lane % P, q = lane / P;
  const float* yj = y + j * a.head_stride;
  const int64_t id = pos0 + j;
  const bool valid = id < a.first + a.n;
  for (int t = 0; t < a.n_textures; ++t) {
    const float* ep = yj + a.ep_off[t];
    const float* col = yj + a.endpoint_dim + a.ch_off[t];
    const float* wt = yj + a.endpoint_dim + t;  // naive: texel tx's weight at wt[tx * n_textures]
    uint64_t bits;
    if (a.formats[t] == NTBC_BC1) {
      const dev::Bc1Pal p = dev::bc1_from_heads(ep, tab);
      uint32_t codes = 0;
      if (a.naive) {
        // stored c0 is the predicted endpoint 1 when the endpoints were swapped: the weight turns round
        const bool swap = dev::rgb565(ep[0], ep[1], ep[2]) < dev::rgb565(ep[3], ep[4], ep[5]);
#pragma unroll
        for (int i = 0; i < TPL; ++i) {
          const int tx = q * TPL + i;
          const float w = wt[tx * a.n_textures];
          float wn;
          const int n = dev::naive_index_bc1(swap ? __fsub_rn(1.0f, w) : w, &wn);
          codes |= ((p.map >> (2 * n)) & 3u) << (2 * tx);
        }
      } else {
#pragma unroll
        for (int i = 0; i < TPL; ++i) {
          const int tx = q * TPL + i;
          const float* c = col + tx * a.channels;
          codes |= dev::bc1_code(p, c[0], c[1], c[2]) << (2 * tx);
        }
      }
#pragma unroll
      for (int o = P; o < 64; o <<= 1) codes |= __shfl_xor(codes, o);
      bits = (uint64_t)p.c0 | ((uint64_t)p.c1 << 16) | ((uint64_t)codes << 32);
    } else {
      const dev::Bc4Pal p = dev::bc4_from_heads(ep, tab);
      uint64_t codes = 0;
#pragma unroll
      for (int i = 0; i < TPL; ++i) {
        const int tx = q * TPL + i;
        uint32_t code;
        if (a.naive) {
          float wn;
          code = (p.map >> (3 * dev::naive_index_bc4(wt[tx * a.n_textures], p.eight, &wn))) & 7u;
        } else {
          code = dev::bc4_code(p, col[tx * a.channels]);
        }
        codes |= (uint64_t)code << (3 * tx);
      }
#pragma unroll
      for (int o = P; o < 64; o <<= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)codes, o);
        const uint32_t hi = __shfl_xor((uint32_t)(codes >> 32), o);
        codes |= ((uint64_t)hi << 32) | lo;
      }
      bits = (uint64_t)p.e0 | ((uint64_t)p.e1 << 8) | (codes << 16);
    }
    if (q == 0 && valid) a.out[(int64_t)t * a.n + (id - a.first)] = bits;
  }
  if (a.heads) {
    for (int e = lane; e < P * a.head_dim; e += 64) {
      const int jj = e / a.head_dim, k = e % a.head_dim;
      const int64_t idj = pos0 + jj;
      if (idj < a.first + a.n) a.heads[(idj - a.first) * a.head_dim + k] = y[jj * a.head_stride + k];
    }
  }
}

// ------------------------------------------------------------------------------ 16-bit kernel
template <Lp L, int HID>
__global__ void __launch_bounds__(64 * kWaves) k_infer_lp(InferArgs a) {
  constexpr int S = HID / 16;  // K-steps of a hidden input
  constexpr int T = HID / 32;  // output tiles of a hidden layer
  constexpr int TC = T < 4 ? T : 4;  // output tiles per pass
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 31, g = lane >> 5;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t pos0 = a.first + (tile * kWaves + wave) * 32;
  const int64_t last = a.first + a.n - 1;
  const int64_t id = pos0 + j <= last ? pos0 + j : last;
  const int bx = (int)(id % a.grid.blocks_w), by = (int)(id / a.grid.blocks_w);

  u32x4 bin[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    float v[8];
    if (s < a.ksteps[0]) {
      dev::features<8>(a.grid, 16 * s + 8 * g, bx, by, v);
    } else {
#pragma unroll
      for (int m = 0; m < 8; ++m) v[m] = 0.0f;
    }
    bin[s] = x8_of<L>(v);
  }

  const u32x4* wp = reinterpret_cast<const u32x4*>(a.wpack);
  // hidden layers
  for (int layer = 0; layer < a.n_layers - 1; ++layer) {
    const int ks = a.ksteps[layer];
    const u32x4* wl = wp + a.pack_off[layer];
    const float* bl = a.bias + a.bias_off[layer];
    u32x4 bout[S];
#pragma unroll
    for (int t0 = 0; t0 < T; t0 += TC) {
      f32x16_t acc[TC];
#pragma unroll
      for (int u = 0; u < TC; ++u) acc[u] = f32x16_t{};
#pragma unroll
      for (int s = 0; s < S; ++s) {
        if (s < ks) {
#pragma unroll
          for (int u = 0; u < TC; ++u) {
            acc[u] = mfma16<L>(wl[((int64_t)(t0 + u) * ks + s) * 64 + lane], bin[s], acc[u]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < TC; ++u) {
        const int t = t0 + u;
        float r[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int neuron = 32 * t + 8 * (v / 4) + 4 * g + (v % 4);
          r[v] = fmaxf(acc[u][v] + bl[neuron], 0.0f);
        }
        bout[2 * t] = x8_of<L>(r);
        bout[2 * t + 1] = x8_of<L>(r + 8);
      }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) bin[s] = bout[s];
  }
  // head layer: sigmoid outputs into LDS
  float* y = lds + wave * 32 * a.head_stride;
  {
    const int layer = a.n_layers - 1;
    const int ks = a.ksteps[layer];
    const u32x4* wl = wp + a.pack_off[layer];
    const float* bl = a.bias + a.bias_off[layer];
    for (int t0 = 0; t0 < a.otiles[layer]; t0 += 2) {
      f32x16_t acc[2] = {f32x16_t{}, f32x16_t{}};
      const int nt = a.otiles[layer] - t0 < 2 ? 1 : 2;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        if (s < ks) {
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            if (u < nt) {
              acc[u] = mfma16<L>(wl[((int64_t)(t0 + u) * ks + s) * 64 + lane], bin[s], acc[u]);
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (u < nt) {
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int neuron = 32 * (t0 + u) + 8 * (v / 4) + 4 * g + (v % 4);
            if (neuron < a.head_dim) y[j * a.head_stride + neuron] = sigmoid(acc[u][v] + bl[neuron]);
          }
        }
      }
    }
  }
  __syncthreads();
  pack_blocks<32>(a, y, lane, pos0);
}

// ------------------------------------------------------------------------------ 16-bit kernel, LDS-staged
// kLdsWaves waves of 32 block positions each share every weight chunk: a chunk is kChunkTiles output
// tiles of one layer over the layer's full K, copied global -> LDS (direct DMA) one chunk ahead of
// its use (double buffer).  The block is sized so that two blocks fit in a CU's LDS (two waves per
// SIMD, 256 registers each; the staged heads reuse the chunk buffers): while one block is in its
// VALU-heavy phases (grid gather, sigmoid, BC packing), the other keeps the matrix cores busy.  The per-value work between the matrix products is
// a few instructions: biases come from LDS, conversion to the 16-bit format is one packed convert
// (round to nearest even) and the ReLU is a packed 16-bit integer max on the pairs.  The head layer
// keeps its accumulators in registers and applies the sigmoid there; the heads are staged in LDS in
// two halves of 16 positions per wave for the BC epilogue, which reads code/255 from an LDS table.
constexpr int kHeadTiles = 6;
static_assert(32 * kHeadTiles == kHeadRows, "head rows");
// chunks of the deepest network (kMaxLayers layers): FP32 (one 16-row tile per chunk, width 256)
// needs 4 * 16 + 12 = 76, the 16-bit formats (two 32-row tiles) 4 * 4 + 3
constexpr int kMaxChunks = 80;
constexpr int kLdsWaves = 4;
constexpr int kChunkTiles = 2;

// Direct global -> LDS copy of a weight chunk (global_load_lds_dwordx4): element e = tid + NT*r goes
// to dst[e]; within a wave the 64 lanes write 64 consecutive 16-byte slots from the wave's LDS base.
// The copy completes at the next s_waitcnt vmcnt(0).
// A wave-uniform pointer made opaque to the optimizer (kept in scalar registers), so that a load from
// it plus a 32-bit lane offset uses the scalar-base form instead of a per-lane 64-bit address.
__device__ __forceinline__ const char* scalar_ptr(const void* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<const char*>(((uint64_t)hi << 32) | lo);
}

template <int PR, int NT>
__device__ __forceinline__ void chunk_dma(const u32x4* __restrict__ wp, int64_t src, int len, u32x4* dst, int tid) {
  const int wave_base = __builtin_amdgcn_readfirstlane(tid & ~63);
  if (len == PR * NT) {
    // a full chunk (the usual case, uniform): no per-slot bounds test, the same per-lane byte offset
    // for every slot, the slot's global base and LDS destination are scalars
    const uint32_t voff = (uint32_t)tid * 16u;
#pragma unroll
    for (int r = 0; r < PR; ++r)
      __builtin_amdgcn_global_load_lds(scalar_ptr(wp + src + NT * r) + voff,
                                       (__attribute__((address_space(3))) void*)(dst + wave_base + NT * r), 16, 0, 0);
    return;
  }
#pragma unroll
  for (int r = 0; r < PR; ++r) {
    const int e = tid + NT * r;
    if (e < len)
      __builtin_amdgcn_global_load_lds(wp + src + e, (__attribute__((address_space(3))) void*)(dst + wave_base + NT * r),
                                       16, 0, 0);
  }
}

__device__ __forceinline__ void wait_dma() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

struct ChunkTable {
  int n;
  int64_t src[kMaxChunks];  // u32x4 offset in the packed weights
  int len[kMaxChunks];      // u32x4 count
  int n_bias;               // padded biases of all layers (floats, a multiple of 4)
  int stage;                // u32x4 slots of the staging area: the two chunk buffers, later the heads
};

// Start value of a tile's accumulators: the bias of its neurons (bias4[q] = neurons 32t + 8q + 4g .. +3,
// the accumulator layout) for the 16-bit formats, so the products add onto it; zero for FP8, whose
// products are rescaled before the bias is added.
template <Lp L>
__device__ __forceinline__ f32x16_t acc_init(const float* bt, int g) {
  f32x16_t r{};
  if constexpr (L != Lp::FP8) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 b = *reinterpret_cast<const float4*>(bt + 8 * q + 4 * g);
      r[4 * q] = b.x;
      r[4 * q + 1] = b.y;
      r[4 * q + 2] = b.z;
      r[4 * q + 3] = b.w;
    }
  }
  return r;
}

// ReLU and conversion of a tile's accumulators (which started from the bias): the two B-operand words
// of K-steps 2t and 2t+1 of the next layer.  FP8: z = acc * (s_x s_w) + b (bias4[q] = the four
// consecutive neurons 32t + 8q + 4g .. +3), then the ReLU output is divided by the next layer's s_x
// (`mul`, `inv_next`: exact powers of two).
template <Lp L>
__device__ __forceinline__ void hidden_epilogue(const f32x16_t& acc, const float* bt, int g, typename LpOp<L>::type* lo,
                                                typename LpOp<L>::type* hi, float mul, float inv_next) {
  if constexpr (L == Lp::FP8) {
    float r[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 b = *reinterpret_cast<const float4*>(bt + 8 * q + 4 * g);
      const float bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float z = acc[4 * q + k] * mul + bv[k];
        r[4 * q + k] = (z < 0.0f ? 0.0f : z) * inv_next;
      }
    }
    *lo = x8_of<L>(r);
    *hi = x8_of<L>(r + 8);
  } else {
    uint32_t w[8];  // the accumulators started from the bias (acc_init)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      w[2 * q] = relu16x2(cvt2<L>(acc[4 * q], acc[4 * q + 1]));
      w[2 * q + 1] = relu16x2(cvt2<L>(acc[4 * q + 2], acc[4 * q + 3]));
    }
    *lo = mk4(w[0], w[1], w[2], w[3]);
    *hi = mk4(w[4], w[5], w[6], w[7]);
  }
}

// FP8 E4M3 mode takes bfloat16 operands in the first layer and the head and E4M3 operands in the
// middle hidden layers.  First layer -> middle: the bias-initialised accumulators, ReLU, divided by the
// next layer's s_x (an exact power of two), rounded to E4M3.
__device__ __forceinline__ void epi_bf16_to_fp8(const f32x16_t& acc, u32x2* lo, u32x2* hi, float inv_next) {
  float r[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const float z = acc[v];
    r[v] = (z < 0.0f ? 0.0f : z) * inv_next;
  }
  *lo = x8_of<Lp::FP8>(r);
  *hi = x8_of<Lp::FP8>(r + 8);
}

// Last middle layer -> head: z = acc * (s_x s_w) + b, ReLU, rounded to bfloat16 (bias4[q] = the four
// consecutive neurons 32t + 8q + 4g .. +3).
__device__ __forceinline__ void epi_fp8_to_bf16(const f32x16_t& acc, const float* bt, int g, u32x4* lo, u32x4* hi,
                                                float mul) {
  float r[16];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 b = *reinterpret_cast<const float4*>(bt + 8 * q + 4 * g);
    const float bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float z = acc[4 * q + k] * mul + bv[k];
      r[4 * q + k] = z < 0.0f ? 0.0f : z;
    }
  }
  *lo = x8_of<Lp::BF16>(r);
  *hi = x8_of<Lp::BF16>(r + 8);
}

// One chunk of a layer: output tiles tc*CT .. tc*CT+CT-1 (those below `valid`) over KS K-steps, the
// A fragments read from LDS kPrefetch K-steps ahead of their product.
constexpr int kPrefetch = 4;

template <Lp L, int KS, int CT, int S>
__device__ __forceinline__ void chunk_mfma(const typename LpOp<L>::type* wb, int ks_stride,
                                           const typename LpOp<L>::type (&b)[S], int lane, int valid,
                                           f32x16_t (&acc)[CT]) {
  typedef typename LpOp<L>::type Op;
  constexpr int PD = kPrefetch < KS ? kPrefetch : KS;
  Op ring[PD][CT];
#pragma unroll
  for (int d = 0; d < PD; ++d)
#pragma unroll
    for (int u = 0; u < CT; ++u) ring[d][u] = u < valid ? wb[(u * ks_stride + d) * 64 + lane] : Op{};
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    Op cur[CT];
#pragma unroll
    for (int u = 0; u < CT; ++u) cur[u] = ring[s % PD][u];
    if (s + PD < KS) {
#pragma unroll
      for (int u = 0; u < CT; ++u)
        if (u < valid) ring[s % PD][u] = wb[(u * ks_stride + s + PD) * 64 + lane];
    }
#pragma unroll
    for (int u = 0; u < CT; ++u)
      if (u < valid) acc[u] = mfma16<L>(cur[u], b[s], acc[u]);
    __builtin_amdgcn_sched_barrier(0);  // A fragments are read PD K-steps ahead, no further
  }
}

// Per-layer FP8 factors: mul[k] = s_x s_w rescales layer k's products, inv[k] = 1 / s_x divides its
// input (both exact: the scales are powers of two).  Unused (1) for the 16-bit formats.
struct Fp8Factors {
  float mul[kMaxLayers], inv[kMaxLayers + 1];
};

template <Lp L>
__device__ __forceinline__ Fp8Factors fp8_factors(const InferArgs& a) {
  Fp8Factors f;
#pragma unroll
  for (int k = 0; k < kMaxLayers; ++k) {
    const bool on = L == Lp::FP8 && k < a.n_layers;
    f.mul[k] = on ? a.fp8_scales[2 * k] * a.fp8_scales[2 * k + 1] : 1.0f;
    f.inv[k] = on ? 1.0f / a.fp8_scales[2 * k] : 1.0f;
  }
  f.inv[kMaxLayers] = 1.0f;
  return f;
}

// One middle hidden layer: every chunk (CT output tiles over the full K) through the matrix cores,
// bias + ReLU + conversion into `out`; the next chunk's DMA runs under the products.
template <Lp L, int S, int T, int CT, int PR, int NT, int CH>
__device__ __forceinline__ void hidden_layer(const typename LpOp<L>::type (&in)[S], typename LpOp<L>::type (&out)[S],
                                             const float* bl, float mul, float inv_next, const u32x4* __restrict__ wp,
                                             const ChunkTable& ct, u32x4* smem, int& c, int tid, int lane, int g) {
  typedef typename LpOp<L>::type Op;
#pragma unroll
  for (int tc = 0; tc < T / CT; ++tc) {
    if (c + 1 < ct.n) chunk_dma<PR, NT>(wp, ct.src[c + 1], ct.len[c + 1], smem + ((c + 1) & 1) * CH, tid);
    f32x16_t acc[CT];
#pragma unroll
    for (int u = 0; u < CT; ++u) acc[u] = acc_init<L>(bl + 32 * (CT * tc + u), g);
    chunk_mfma<L, S, CT, S>(reinterpret_cast<const Op*>(smem + (c & 1) * CH), S, in, lane, CT, acc);
#pragma unroll
    for (int u = 0; u < CT; ++u) {
      const int t = CT * tc + u;
      hidden_epilogue<L>(acc[u], bl + 32 * t, g, &out[2 * t], &out[2 * t + 1], mul, inv_next);
    }
    wait_dma();
    __syncthreads();
    ++c;
  }
}

// The last middle hidden layer of FP8 mode: E4M3 products, outputs rounded to bfloat16 for the head.
template <int S, int T, int CT, int PR, int NT, int CH>
__device__ __forceinline__ void last_middle_fp8(const u32x2 (&in)[S], u32x4 (&out)[S], const float* bl, float mul,
                                                const u32x4* __restrict__ wp, const ChunkTable& ct, u32x4* smem, int& c,
                                                int tid, int lane, int g) {
#pragma unroll
  for (int tc = 0; tc < T / CT; ++tc) {
    if (c + 1 < ct.n) chunk_dma<PR, NT>(wp, ct.src[c + 1], ct.len[c + 1], smem + ((c + 1) & 1) * CH, tid);
    f32x16_t acc[CT];
#pragma unroll
    for (int u = 0; u < CT; ++u) acc[u] = f32x16_t{};
    chunk_mfma<Lp::FP8, S, CT, S>(reinterpret_cast<const u32x2*>(smem + (c & 1) * CH), S, in, lane, CT, acc);
#pragma unroll
    for (int u = 0; u < CT; ++u) {
      const int t = CT * tc + u;
      epi_fp8_to_bf16(acc[u], bl + 32 * t, g, &out[2 * t], &out[2 * t + 1], mul);
    }
    wait_dma();
    __syncthreads();
    ++c;
  }
}

// Register-resident BC epilogue.  Lane (j, g) of a wave holds, after the head products, accumulator
// v of head tile t = packed head row 32t + 8(v/4) + 4g + v%4 of position j; call 16t + v the lane's
// slot.  The host permutes the head rows (weights and biases) so that, with NB1 BC1 and NB4 BC4
// textures (BC1 first in slot order), lane group g holds for every texture the predicted colours of
// texels 8g .. 8g+7 and endpoint g:
//   BC1 texture k: colour channel c of texel 8g+i at slot 24k + 3i + c, endpoint g (R, G, B) at kE1 + 3k + c
//   BC4 texture k: texel 8g+i at slot kC4 + 8k + i, endpoint g at kE4 + k
// (27 NB1 + 9 NB4 = head_dim / 2 slots).  The two lanes of a position exchange their quantised
// endpoint g and their half of the index bits with one lane swap each, so the BC words are made
// without staging the heads in LDS, and each palette is built by two lanes instead of four.
template <int NB1, int NB4>
struct RegLayout {
  static constexpr int kC4 = 24 * NB1;
  static constexpr int kE1 = kC4 + 8 * NB4;
  static constexpr int kE4 = kE1 + 3 * NB1;
  static constexpr int kUsed = kE4 + NB4;
  static_assert(NB1 <= 2 && NB4 <= 4 && kUsed <= 16 * kHeadTiles, "slot layout");
};

// Canonical head neuron of slot `slot` in lane group g (the inverse of the host's row permutation).
template <int NB1, int NB4, typename ArgsT>
__device__ __forceinline__ int reg_canonical(ArgsT a, int slot, int g) {
  using Y = RegLayout<NB1, NB4>;
  if (slot < Y::kC4) return a.endpoint_dim + (8 * g + (slot % 24) / 3) * a.channels + a.reg_ch[slot / 24] + slot % 3;
  if (slot < Y::kE1) return a.endpoint_dim + (8 * g + (slot - Y::kC4) % 8) * a.channels + a.reg_ch[NB1 + (slot - Y::kC4) / 8];
  if (slot < Y::kE4) return a.reg_ep[(slot - Y::kE1) / 3] + 3 * g + (slot - Y::kE1) % 3;
  return a.reg_ep[NB1 + slot - Y::kE4] + g;
}

template <int NB1, int NB4, typename ArgsT>
__device__ __forceinline__ void reg_epilogue(ArgsT a, const f32x16_t (&h)[kHeadTiles], const float* tab, int g,
                                             int64_t id, bool valid) {
  using Y = RegLayout<NB1, NB4>;
#define NTBC_SLOT(x) h[(x) / 16][(x) % 16]
  // value of the partner lane (lane ^ 32): one LDS-crossbar permute with a fixed address
  const int partner = (((int)threadIdx.x & 63) ^ 32) << 2;
  auto swap = [partner](uint32_t v) { return (uint32_t)__builtin_amdgcn_ds_bpermute(partner, (int)v); };
  // endpoint g of every texture, quantised here; the partner lane (lane ^ 32) holds the other one
  uint32_t w1 = 0, w4 = 0;
#pragma unroll
  for (int k = 0; k < NB1; ++k)
    w1 |= dev::rgb565(NTBC_SLOT(Y::kE1 + 3 * k), NTBC_SLOT(Y::kE1 + 3 * k + 1), NTBC_SLOT(Y::kE1 + 3 * k + 2)) << (16 * k);
#pragma unroll
  for (int k = 0; k < NB4; ++k) w4 |= (uint32_t)dev::quant_bits(NTBC_SLOT(Y::kE4 + k), 255.0f) << (8 * k);
  const uint32_t o1 = NB1 > 0 ? swap(w1) : 0u;
  const uint32_t o4 = NB4 > 0 ? swap(w4) : 0u;
  const uint32_t a1 = g ? o1 : w1, b1 = g ? w1 : o1;  // endpoint 0 / endpoint 1 words
  const uint32_t a4 = g ? o4 : w4, b4 = g ? w4 : o4;
  const int64_t row = id - a.first;
#pragma unroll
  for (int k = 0; k < NB1; ++k) {
    const dev::Bc1Pal p = dev::bc1_palette((a1 >> (16 * k)) & 0xFFFFu, (b1 >> (16 * k)) & 0xFFFFu, tab);
    uint32_t codes = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      codes |= dev::bc1_code(p, NTBC_SLOT(24 * k + 3 * i), NTBC_SLOT(24 * k + 3 * i + 1), NTBC_SLOT(24 * k + 3 * i + 2))
               << (2 * i);
    const uint32_t hi = swap(codes);  // texels 8..15 from lane group 1
    if (g == 0 && valid)
      a.out[(int64_t)a.reg_tex[k] * a.n + row] = (uint64_t)p.c0 | ((uint64_t)p.c1 << 16) | ((uint64_t)(codes | (hi << 16)) << 32);
  }
#pragma unroll
  for (int k = 0; k < NB4; ++k) {
    const dev::Bc4Pal p = dev::bc4_palette((int)((a4 >> (8 * k)) & 255u), (int)((b4 >> (8 * k)) & 255u), tab);
    uint32_t codes = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) codes |= dev::bc4_code(p, NTBC_SLOT(Y::kC4 + 8 * k + i)) << (3 * i);
    const uint32_t hi = swap(codes);
    if (g == 0 && valid)
      a.out[(int64_t)a.reg_tex[NB1 + k] * a.n + row] =
          (uint64_t)p.e0 | ((uint64_t)p.e1 << 8) | (((uint64_t)codes | ((uint64_t)hi << 24)) << 16);
  }
  if (a.heads && valid) {
    float* hr = a.heads + row * a.head_dim;
#pragma unroll
    for (int x = 0; x < Y::kUsed; ++x) hr[reg_canonical<NB1, NB4>(a, x, g)] = NTBC_SLOT(x);
  }
#undef NTBC_SLOT
}

// The head's input: the last hidden layer's operands, which FP8 mode rounds to bfloat16 separately.
template <bool MIX, typename A, typename B>
__device__ __forceinline__ const B& pick_head_input(const A& bin, const B& hb) {
  if constexpr (MIX)
    return hb;
  else
    return bin;
}

// The fused network of one tile of W * 32 block positions (W waves; tile index `tile` of the range
// a.first .. a.first + a.n).
// ArgsT/ChunksT: by value for the single-range kernel (its by-value parameters are then read in place
// from the kernel-argument segment), references for work items in device memory.
template <Lp L, int HID, int KS0, int NH, int NB1 = -1, int NB4 = 0, typename ArgsT = const InferArgs,
          typename ChunksT = const ChunkTable, int W = kLdsWaves>
__device__ __forceinline__ void infer_tile(ArgsT a, ChunksT ct, int64_t tile) {
  // FP8 mode (MIX): E4M3 operands in the middle hidden layers (Op), bfloat16 in the first layer and the
  // head (OpE); the other formats use one operand type throughout (OpE = Op)
  constexpr bool MIX = L == Lp::FP8;
  constexpr Lp LE = MIX ? Lp::BF16 : L;
  typedef typename LpOp<L>::type Op;
  typedef typename LpOp<LE>::type OpE;
  constexpr int S = HID / 16;
  constexpr int T = HID / 32;
  constexpr int CT = kChunkTiles;
  constexpr int CH = CT * S * 64 * (int)sizeof(OpE) / 16;  // u32x4 per chunk buffer (the wider operand)
  constexpr int NT = 64 * W;                            // threads
  constexpr int PR = (CH + NT - 1) / NT;                // DMA slots per thread
  static_assert(T % CT == 0 && kHeadTiles % CT == 0, "chunk tiles must divide the tile counts");
  extern __shared__ u32x4 smem[];
  float* tab = reinterpret_cast<float*>(smem + ct.stage);
  float* bias_s = tab + 256;
  float* ybase = reinterpret_cast<float*>(smem);  // the heads reuse the chunk buffers after the last chunk
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int j = lane & 31, g = lane >> 5;
  const int64_t pos0 = a.first + (tile * W + wave) * 32;
  const int64_t last = a.first + a.n - 1;
  const int64_t id = pos0 + j <= last ? pos0 + j : last;
  const int bx = (int)(id % a.grid.blocks_w), by = (int)(id / a.grid.blocks_w);
  const u32x4* wp = reinterpret_cast<const u32x4*>(a.wpack);
  const Fp8Factors f8 = fp8_factors<L>(a);

  chunk_dma<PR, NT>(wp, ct.src[0], ct.len[0], smem, tid);
  for (int i = tid; i < 256; i += NT) tab[i] = (float)i / 255.0f;
  for (int i = tid; i < ct.n_bias; i += NT) bias_s[i] = a.bias[i];

  // grid features: the first layer's B operands
  OpE x0[KS0];
#pragma unroll
  for (int s = 0; s < KS0; ++s) {
    float v[8];
    dev::features<8>(a.grid, 16 * s + 8 * g, bx, by, v);
    x0[s] = x8_of<LE>(v);
  }
  wait_dma();
  __syncthreads();

  int c = 0;
  Op bin[S], bout[S];
  {
    const float* bl = bias_s + a.bias_off[0];
#pragma unroll
    for (int tc = 0; tc < T / CT; ++tc) {
      if (c + 1 < ct.n) chunk_dma<PR, NT>(wp, ct.src[c + 1], ct.len[c + 1], smem + ((c + 1) & 1) * CH, tid);
      f32x16_t acc[CT];
#pragma unroll
      for (int u = 0; u < CT; ++u) acc[u] = acc_init<LE>(bl + 32 * (CT * tc + u), g);
      chunk_mfma<LE, KS0, CT, KS0>(reinterpret_cast<const OpE*>(smem + (c & 1) * CH), KS0, x0, lane, CT, acc);
#pragma unroll
      for (int u = 0; u < CT; ++u) {
        const int t = CT * tc + u;
        if constexpr (MIX)
          epi_bf16_to_fp8(acc[u], &bin[2 * t], &bin[2 * t + 1], f8.inv[1]);
        else
          hidden_epilogue<L>(acc[u], bl + 32 * t, g, &bin[2 * t], &bin[2 * t + 1], f8.mul[0], f8.inv[1]);
      }
      wait_dma();
      __syncthreads();
      ++c;
    }
  }
  // middle hidden layers: NH of them unrolled at compile time (the two register arrays alternate, so
  // nothing is copied), or NH < 0: a run-time count.  FP8 mode: the last one rounds its outputs to
  // bfloat16 for the head (hb); FP8 needs at least one middle layer (the host checks).
  OpE hb[S];  // FP8 mode only (unused, and removed by the compiler, otherwise)
  if constexpr (MIX) {
    if constexpr (NH >= 0) {
      static_assert(NH >= 1 && NH <= 2, "one or two unrolled middle layers");
      if constexpr (NH == 2) {
        hidden_layer<L, S, T, CT, PR, NT, CH>(bin, bout, bias_s + a.bias_off[1], f8.mul[1], f8.inv[2], wp, ct, smem, c,
                                              tid, lane, g);
        last_middle_fp8<S, T, CT, PR, NT, CH>(bout, hb, bias_s + a.bias_off[2], f8.mul[2], wp, ct, smem, c, tid, lane, g);
      } else {
        last_middle_fp8<S, T, CT, PR, NT, CH>(bin, hb, bias_s + a.bias_off[1], f8.mul[1], wp, ct, smem, c, tid, lane, g);
      }
    } else {
      for (int layer = 1; layer < a.n_layers - 2; ++layer) {
        const float mul = a.fp8_scales[2 * layer] * a.fp8_scales[2 * layer + 1];
        const float inv_next = 1.0f / a.fp8_scales[2 * layer + 2];
        hidden_layer<L, S, T, CT, PR, NT, CH>(bin, bout, bias_s + a.bias_off[layer], mul, inv_next, wp, ct, smem, c, tid,
                                              lane, g);
#pragma unroll
        for (int s = 0; s < S; ++s) bin[s] = bout[s];
      }
      const int layer = a.n_layers - 2;
      last_middle_fp8<S, T, CT, PR, NT, CH>(bin, hb, bias_s + a.bias_off[layer],
                                            a.fp8_scales[2 * layer] * a.fp8_scales[2 * layer + 1], wp, ct, smem, c, tid,
                                            lane, g);
    }
  } else if constexpr (NH >= 0) {
    static_assert(NH <= 2, "at most two unrolled middle layers");
    if constexpr (NH >= 1)
      hidden_layer<L, S, T, CT, PR, NT, CH>(bin, bout, bias_s + a.bias_off[1], f8.mul[1], f8.inv[2], wp, ct, smem, c,
                                            tid, lane, g);
    if constexpr (NH >= 2)
      hidden_layer<L, S, T, CT, PR, NT, CH>(bout, bin, bias_s + a.bias_off[2], f8.mul[2], f8.inv[3], wp, ct, smem, c,
                                            tid, lane, g);
    if constexpr (NH == 1) {
#pragma unroll
      for (int s = 0; s < S; ++s) bin[s] = bout[s];
    }
  } else {
    for (int layer = 1; layer < a.n_layers - 1; ++layer) {
      hidden_layer<L, S, T, CT, PR, NT, CH>(bin, bout, bias_s + a.bias_off[layer], 1.0f, 1.0f, wp, ct, smem, c, tid,
                                            lane, g);
#pragma unroll
      for (int s = 0; s < S; ++s) bin[s] = bout[s];
    }
  }
  const OpE (&hin)[S] = pick_head_input<MIX>(bin, hb);
  // head layer, accumulators kept for the BC epilogue
  const int head = a.n_layers - 1;
  const int nht = a.otiles[head];
  const float* bl = bias_s + a.bias_off[head];
  f32x16_t hacc[kHeadTiles];
#pragma unroll
  for (int t = 0; t < kHeadTiles; ++t) hacc[t] = f32x16_t{};
#pragma unroll
  for (int tc = 0; tc < kHeadTiles / CT; ++tc) {
    if (CT * tc < nht) {
      if (c + 1 < ct.n) chunk_dma<PR, NT>(wp, ct.src[c + 1], ct.len[c + 1], smem + ((c + 1) & 1) * CH, tid);
      f32x16_t acc[CT];
#pragma unroll
      for (int u = 0; u < CT; ++u) acc[u] = CT * tc + u < nht ? acc_init<LE>(bl + 32 * (CT * tc + u), g) : f32x16_t{};
      chunk_mfma<LE, S, CT, S>(reinterpret_cast<const OpE*>(smem + (c & 1) * CH), S, hin, lane, nht - CT * tc, acc);
#pragma unroll
      for (int u = 0; u < CT; ++u) hacc[CT * tc + u] = acc[u];
      wait_dma();
      __syncthreads();
      ++c;
    }
  }
  // sigmoid heads in registers (all lanes; the register epilogue's layout uses the first kUsed slots)
  constexpr int used = NB1 >= 0 ? RegLayout<NB1 < 0 ? 0 : NB1, NB4>::kUsed : 16 * kHeadTiles;
#pragma unroll
  for (int t = 0; t < kHeadTiles; ++t) {
    if (t < nht) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (16 * t + 4 * q >= used) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (16 * t + 4 * q + r >= used) continue;
          hacc[t][4 * q + r] = sigmoid_fast(hacc[t][4 * q + r]);  // the bias is in the accumulators
        }
      }
    }
  }
  if constexpr (NB1 >= 0) {
    reg_epilogue<NB1, NB4>(a, hacc, tab, g, id, pos0 + j <= last);
    return;
  }
  // otherwise staged in LDS 16 positions at a time for the pack
  float* y = ybase + wave * 16 * a.head_stride;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    if ((j >> 4) == half) {
#pragma unroll
      for (int t = 0; t < kHeadTiles; ++t) {
        if (t < nht) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int n0 = 32 * t + 8 * q + 4 * g;
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (n0 + r < a.head_dim) y[(j & 15) * a.head_stride + n0 + r] = hacc[t][4 * q + r];
          }
        }
      }
    }
    __syncthreads();
    pack_blocks<16>(a, y, lane, pos0 + 16 * half, tab);
    __syncthreads();
  }
}

// One block range per launch, its arguments in the kernel-argument segment.
template <Lp L, int HID, int KS0, int NH, int NB1, int NB4>
__global__ void __launch_bounds__(64 * kLdsWaves) __attribute__((amdgpu_waves_per_eu(2)))
k_infer_lds(InferArgs a, ChunkTable ct) {
  infer_tile<L, HID, KS0, NH, NB1, NB4>(a, ct, xcd_tile(blockIdx.x, gridDim.x));
}

// ------------------------------------------------------------------------------ launch over work items
// Many block ranges (materials, their mip levels) in one launch per kernel instance.  The items live
// in device memory (their arguments are read through the scalar cache, and
// arrays in them may be indexed at run time without private copies): item i owns the tiles
// [tile_begin, tile_begin + tiles) of the launch; a block takes tile xcd_tile(blockIdx) (consecutive
// tiles on one XCD), finds its item by binary search over tile_begin (uniform), runs the tile, and
// the last block of an item to finish stamps the item's completion time (the 100 MHz real-time
// counter) when stamps are requested.
struct BatchItem {
  InferArgs a;
  ChunkTable ct;
  int64_t tile_begin, tiles;
  int32_t index;  // position of the item in the caller's list (stamps)
};

template <Lp L, int HID, int KS0, int NH, int NB1, int NB4, int W>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(2)))
k_infer_lds_batch(const BatchItem* __restrict__ items, int n_items, unsigned* __restrict__ done,
                  uint64_t* __restrict__ stamps) {
  // the items are read-only for the whole launch: reading them through the constant address space
  // lets the compiler keep the arguments in scalar registers and reuse them across the kernel's stores
  typedef const __attribute__((address_space(4))) BatchItem ConstItem;
  const ConstItem* citems = (const ConstItem*)items;
  const int64_t b = xcd_tile(blockIdx.x, gridDim.x);
  int lo = 0, hi = n_items - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (citems[mid].tile_begin <= b) lo = mid;
    else hi = mid - 1;
  }
  const BatchItem& it = *(const BatchItem*)(citems + lo);
  infer_tile<L, HID, KS0, NH, NB1, NB4, const InferArgs&, const ChunkTable&, W>(it.a, it.ct, b - it.tile_begin);
  if (stamps != nullptr) {
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      if (atomicAdd(&done[it.index], 1u) + 1u == (unsigned)it.tiles) stamps[1 + it.index] = wall_clock64();
    }
  }
}

__global__ void k_batch_start(unsigned* __restrict__ done, int n, uint64_t* __restrict__ stamps) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) done[i] = 0u;
  if (threadIdx.x == 0 && stamps != nullptr) stamps[0] = wall_clock64();
}

// ------------------------------------------------------------------------------ FP32 kernel
// CALIB: FP8 calibration pass over the sample ids i * stride (i < n): records max |input| of every
// layer (float bits; non-negative floats order like their bits) and stops before the heads.
__device__ __forceinline__ void record_max(unsigned* slot, float m) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) atomicMax(slot, __float_as_uint(m));
}

template <int HID, bool CALIB>
__global__ void __launch_bounds__(64 * kWaves) k_infer_f32(InferArgs a) {
  constexpr int S = HID / 4;   // K-steps (of 4) of a hidden input
  constexpr int T = HID / 16;  // output tiles of a hidden layer
  constexpr int TC = T < 4 ? T : 4;
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t pos0 = a.first + (tile * kWaves + wave) * 16;
  const int64_t last = a.first + a.n - 1;
  int64_t id = pos0 + j <= last ? pos0 + j : last;
  if constexpr (CALIB) id *= a.stride;  // first = 0: sample index -> block id
  const int bx = (int)(id % a.grid.blocks_w), by = (int)(id / a.grid.blocks_w);

  float bin[S];
  float m_in = 0.0f;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    float v[1] = {0.0f};
    if (s < a.ksteps[0]) dev::features<1>(a.grid, 4 * s + g, bx, by, v);
    bin[s] = v[0];
    m_in = fmaxf(m_in, fabsf(v[0]));
  }
  if constexpr (CALIB) record_max(&a.amax[0], m_in);
  const float* wp = reinterpret_cast<const float*>(a.wpack);
  for (int layer = 0; layer < a.n_layers - 1; ++layer) {
    const int ks = a.ksteps[layer];
    const float* wl = wp + a.pack_off[layer];
    const float* bl = a.bias + a.bias_off[layer];
    float bout[S];
#pragma unroll
    for (int t0 = 0; t0 < T; t0 += TC) {
      f32x4_t acc[TC];
#pragma unroll
      for (int u = 0; u < TC; ++u) acc[u] = f32x4_t{};
#pragma unroll
      for (int s = 0; s < S; ++s) {
        if (s < ks) {
#pragma unroll
          for (int u = 0; u < TC; ++u) {
            const float w = wl[((int64_t)(t0 + u) * ks + s) * 64 + lane];
            acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, bin[s], acc[u], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < TC; ++u) {
        const int t = t0 + u;
#pragma unroll
        for (int v = 0; v < 4; ++v) bout[4 * t + v] = fmaxf(acc[u][v] + bl[16 * t + 4 * g + v], 0.0f);
      }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) bin[s] = bout[s];
    if constexpr (CALIB) {
      float m = 0.0f;
#pragma unroll
      for (int s = 0; s < S; ++s) m = fmaxf(m, bin[s]);
      record_max(&a.amax[layer + 1], m);
    }
  }
  if constexpr (CALIB) return;
  float* y = lds + wave * 16 * a.head_stride;
  {
    const int layer = a.n_layers - 1;
    const int ks = a.ksteps[layer];
    const float* wl = wp + a.pack_off[layer];
    const float* bl = a.bias + a.bias_off[layer];
    for (int t0 = 0; t0 < a.otiles[layer]; t0 += 4) {
      f32x4_t acc[4] = {f32x4_t{}, f32x4_t{}, f32x4_t{}, f32x4_t{}};
      const int nt = min(4, a.otiles[layer] - t0);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        if (s < ks) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (u < nt) {
              const float w = wl[((int64_t)(t0 + u) * ks + s) * 64 + lane];
              acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, bin[s], acc[u], 0, 0, 0);
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (u < nt) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int neuron = 16 * (t0 + u) + 4 * g + v;
            if (neuron < a.head_dim) y[j * a.head_stride + neuron] = sigmoid(acc[u][v] + bl[neuron]);
          }
        }
      }
    }
  }
  __syncthreads();
  pack_blocks<16>(a, y, lane, pos0);
}

// ------------------------------------------------------------------------------ FP32 kernel, LDS-staged
// FP32 operands through v_mfma_f32_16x16x4f32, 16 positions per wave: lane (j, g) holds position j and
// row g of every K-step, accumulator v of output tile t is neuron 16t + 4g + v, which the packer's
// column order (f32_col) makes input row g of K-step 4t + v of the next layer, so a layer's outputs are
// the next layer's B operands in place.  The weights stream through LDS as in the 16-bit kernels
// (chunks of kF32ChunkTiles output tiles over the full K, double-buffered, the next chunk's DMA under
// the current chunk's products, A fragments read kPrefetch K-steps ahead); every index into the
// activation arrays is a compile-time constant, so they stay in registers.  One 16-row tile per chunk
// (16 KB at width 256) keeps a block's LDS near 46 KB, so three blocks of four waves share a CU: three
// waves per SIMD (at most 168 registers: the two activation arrays take 128), which keeps the matrix
// cores busier than two-tile chunks at two waves per SIMD (3.40 against 3.78 ms at the 4096^2
// five-texture workload, the same words).  The first layer takes
// 4 KQ K-steps (16 KQ inputs; the plan rounds its K-steps up to a multiple of four, padded with zero
// weights).  The heads go through the exact sigmoid into LDS (reusing the chunk buffers) for the pack.
constexpr int kF32Waves = 4;
constexpr int kF32ChunkTiles = 1;
constexpr int kF32HeadTiles = 2 * kHeadTiles;  // 16-row tiles: head_dim <= 192
static_assert(kMaxChunks >= (kMaxLayers - 1) * 16 + kF32HeadTiles, "chunk table of the deepest FP32 network");

template <int KS, int CT, int S>
__device__ __forceinline__ void chunk_mfma_f32(const float* wb, const float (&b)[S], int lane, int valid,
                                               f32x4_t (&acc)[CT]) {
  constexpr int PD = kPrefetch < KS ? kPrefetch : KS;
  float ring[PD][CT];
#pragma unroll
  for (int d = 0; d < PD; ++d)
#pragma unroll
    for (int u = 0; u < CT; ++u) ring[d][u] = u < valid ? wb[(u * KS + d) * 64 + lane] : 0.0f;
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    float cur[CT];
#pragma unroll
    for (int u = 0; u < CT; ++u) cur[u] = ring[s % PD][u];
    if (s + PD < KS) {
#pragma unroll
      for (int u = 0; u < CT; ++u)
        if (u < valid) ring[s % PD][u] = wb[(u * KS + s + PD) * 64 + lane];
    }
#pragma unroll
    for (int u = 0; u < CT; ++u)
      if (u < valid) acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[u], b[s], acc[u], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// One hidden layer of T output tiles over KS input K-steps: bias-initialised accumulators, products,
// ReLU into `out` (K-step 4t + v of the next layer); chunk c is in LDS, chunk c + 1 is fetched meanwhile.
template <int KS, int T, int S, int PR, int NT, int CH>
__device__ __forceinline__ void f32_hidden(const float (&in)[KS], float (&out)[S], const float* bl,
                                           const u32x4* __restrict__ wp, const ChunkTable& ct, u32x4* smem, int& c,
                                           int tid, int lane, int g) {
  constexpr int CT = kF32ChunkTiles;
#pragma unroll
  for (int tc = 0; tc < T / CT; ++tc) {
    if (c + 1 < ct.n) chunk_dma<PR, NT>(wp, ct.src[c + 1], ct.len[c + 1], smem + ((c + 1) & 1) * CH, tid);
    f32x4_t acc[CT];
#pragma unroll
    for (int u = 0; u < CT; ++u) {
      const float4 b = *reinterpret_cast<const float4*>(bl + 16 * (CT * tc + u) + 4 * g);
      acc[u] = f32x4_t{b.x, b.y, b.z, b.w};
    }
    chunk_mfma_f32<KS, CT, KS>(reinterpret_cast<const float*>(smem + (c & 1) * CH), in, lane, CT, acc);
#pragma unroll
    for (int u = 0; u < CT; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) out[4 * (CT * tc + u) + v] = fmaxf(acc[u][v], 0.0f);
    wait_dma();
    __syncthreads();
    ++c;
  }
}

template <int HID, int KQ>
__global__ void __launch_bounds__(64 * kF32Waves) __attribute__((amdgpu_waves_per_eu(3)))
k_infer_f32_lds(InferArgs a, ChunkTable ct) {
  constexpr int S = HID / 4;   // K-steps of a hidden input
  constexpr int T = HID / 16;  // output tiles of a hidden layer
  constexpr int KS0 = 4 * KQ;  // first-layer K-steps
  constexpr int CT = kF32ChunkTiles;
  constexpr int CH = CT * S * 64 / 4;  // u32x4 per chunk buffer
  constexpr int NT = 64 * kF32Waves;
  constexpr int PR = (CH + NT - 1) / NT;
  static_assert(T % CT == 0 && kF32HeadTiles % CT == 0 && KS0 <= S, "tile counts");
  extern __shared__ u32x4 smem[];
  float* tab = reinterpret_cast<float*>(smem + ct.stage);
  float* bias_s = tab + 256;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int64_t pos0 = a.first + (xcd_tile(blockIdx.x, gridDim.x) * kF32Waves + wave) * 16;
  const int64_t last = a.first + a.n - 1;
  const int64_t id = pos0 + j <= last ? pos0 + j : last;
  const int bx = (int)(id % a.grid.blocks_w), by = (int)(id / a.grid.blocks_w);
  const u32x4* wp = reinterpret_cast<const u32x4*>(a.wpack);

  chunk_dma<PR, NT>(wp, ct.src[0], ct.len[0], smem, tid);
  for (int i = tid; i < 256; i += NT) tab[i] = (float)i / 255.0f;
  for (int i = tid; i < ct.n_bias; i += NT) bias_s[i] = a.bias[i];
  float x0[KS0];
#pragma unroll
  for (int s = 0; s < KS0; ++s) dev::features<1>(a.grid, 4 * s + g, bx, by, &x0[s]);
  wait_dma();
  __syncthreads();

  int c = 0;
  float bin[S], bout[S];
  f32_hidden<KS0, T, S, PR, NT, CH>(x0, bin, bias_s + a.bias_off[0], wp, ct, smem, c, tid, lane, g);
  for (int layer = 1; layer < a.n_layers - 1; ++layer) {
    f32_hidden<S, T, S, PR, NT, CH>(bin, bout, bias_s + a.bias_off[layer], wp, ct, smem, c, tid, lane, g);
#pragma unroll
    for (int s = 0; s < S; ++s) bin[s] = bout[s];
  }
  // head: accumulators kept until the last chunk is done, then the sigmoid into the staged heads
  const int head = a.n_layers - 1;
  const int nht = a.otiles[head];
  const float* bl = bias_s + a.bias_off[head];
  f32x4_t hacc[kF32HeadTiles];
#pragma unroll
  for (int tc = 0; tc < kF32HeadTiles / CT; ++tc) {
    if (CT * tc < nht) {
      if (c + 1 < ct.n) chunk_dma<PR, NT>(wp, ct.src[c + 1], ct.len[c + 1], smem + ((c + 1) & 1) * CH, tid);
      f32x4_t acc[CT];
#pragma unroll
      for (int u = 0; u < CT; ++u) {
        const float4 b = *reinterpret_cast<const float4*>(bl + 16 * (CT * tc + u) + 4 * g);
        acc[u] = f32x4_t{b.x, b.y, b.z, b.w};
      }
      chunk_mfma_f32<S, CT, S>(reinterpret_cast<const float*>(smem + (c & 1) * CH), bin, lane, nht - CT * tc, acc);
#pragma unroll
      for (int u = 0; u < CT; ++u) hacc[CT * tc + u] = acc[u];
      wait_dma();
      __syncthreads();
      ++c;
    }
  }
  float* y = reinterpret_cast<float*>(smem) + wave * 16 * a.head_stride;
#pragma unroll
  for (int t = 0; t < kF32HeadTiles; ++t) {
    if (t < nht) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int neuron = 16 * t + 4 * g + v;
        if (neuron < a.head_dim) y[j * a.head_stride + neuron] = sigmoid(hacc[t][v]);
      }
    }
  }
  __syncthreads();
  pack_blocks<16>(a, y, lane, pos0, tab);
}

// ------------------------------------------------------------------------------ host side
constexpr int64_t kCalibBytes = 256;  // 2 x kMaxLayers maxima, padded

struct Plan {
  Shape s;
  int precision;
  int hid_inst;       // kernel instance hidden width (>= shape hidden)
  int rows;           // output-tile rows (32 for 16-bit formats, 16 FP32)
  int kstep;          // K per step (16 for 16-bit formats, 4 FP32)
  int ksteps[kMaxLayers], otiles[kMaxLayers];
  int64_t pack_off[kMaxLayers], bias_off[kMaxLayers];
  int64_t pack_bytes, bias_bytes, total_bytes;
  int64_t calib_offset;  // FP8: FP32 packed weights and per-layer maxima of ntbc_fp8_calibrate
  int positions_per_wave;
};

int make_plan(const ntbc_model_desc* d, int precision, Plan* p) {
  int st = make_shape(d, &p->s);
  if (st != NTBC_OK) return st;
  if (precision != NTBC_FP32 && precision != NTBC_BF16 && precision != NTBC_FP16 && precision != NTBC_FP8_E4M3)
    return fail(NTBC_EINVAL, "precision %d not available for inference", precision);
  if (p->s.n_layers > kMaxLayers) return fail(NTBC_EUNSUPPORTED, "at most %d layers", kMaxLayers);
  p->precision = precision;
  const int h = p->s.hidden;
  p->hid_inst = h <= 64 ? 64 : (h <= 128 ? 128 : 256);
  if (p->s.in_dim > p->hid_inst) return fail(NTBC_EUNSUPPORTED, "in_dim %d > kernel width %d", p->s.in_dim, p->hid_inst);
  const bool bf = precision != NTBC_FP32;  // 32x32x16 matrix shapes (16-bit or FP8 operands)
  p->rows = bf ? 32 : 16;
  p->kstep = bf ? 16 : 4;
  p->positions_per_wave = bf ? 32 : 16;
  const int64_t unit = precision == NTBC_FP8_E4M3 ? 8 : (bf ? 16 : 4);  // bytes per lane operand
  int64_t off = 0, boff = 0;
  for (int k = 0; k < p->s.n_layers; ++k) {
    const int in = k == 0 ? p->s.in_dim : p->hid_inst;
    const int out = k == p->s.n_layers - 1 ? p->s.head_dim : p->hid_inst;
    p->ksteps[k] = (int)ceil_div(in, p->kstep);
    if (!bf && k == 0) p->ksteps[k] = 4 * (int)ceil_div(in, 16);  // whole groups of 16 inputs (zero-padded)
    p->otiles[k] = (int)ceil_div(out, p->rows);
    p->pack_off[k] = off;
    // FP8 mode: offsets in 8-byte units; the first layer and the head hold bfloat16 operands (two units)
    const bool wide = precision == NTBC_FP8_E4M3 && (k == 0 || k == p->s.n_layers - 1);
    off += (int64_t)p->otiles[k] * p->ksteps[k] * 64 * (wide ? 2 : 1);
    p->bias_off[k] = boff;
    boff += (int64_t)p->otiles[k] * p->rows;
  }
  p->pack_bytes = off * unit;
  p->bias_bytes = boff * 4;
  p->total_bytes = ((p->pack_bytes + 255) / 256) * 256 + p->bias_bytes;
  p->calib_offset = -1;
  if (precision == NTBC_FP8_E4M3) {
    // FP8 calibration (ntbc_fp8_calibrate) packs FP32 weights and keeps per-layer maxima after the
    // FP8 area, so a calibration leaves the packed FP8 weights in place
    Plan f;
    const int st32 = make_plan(d, NTBC_FP32, &f);
    if (st32 != NTBC_OK) return st32;
    p->calib_offset = (p->total_bytes + 255) / 256 * 256;
    p->total_bytes = p->calib_offset + f.total_bytes + kCalibBytes;
  }
  return NTBC_OK;
}

// ------------------------------------------------------------------------------ FP8 calibration
struct WMaxArgs {
  const float* w;
  int n_layers;
  int64_t w_off[kMaxLayers], count[kMaxLayers];
  unsigned* amax;  // [kMaxLayers] inputs, then [kMaxLayers] weights (float bits)
};

// max |W| of every layer's weight matrix (its bias excluded); grid (blocks, n_layers).
__global__ void __launch_bounds__(256) k_weight_absmax(WMaxArgs a) {
  const int layer = blockIdx.y;
  float m = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.count[layer];
       i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(a.w[a.w_off[layer] + i]));
  record_max(&a.amax[kMaxLayers + layer], m);
}

__global__ void k_zero_u32(unsigned* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// The smallest power of two s (down to 2^-126) with m / s <= 448; 1 for m = 0 or not finite.  Every
// comparison is exact (448 * 2^e is a float), so the result is a pure function of m.
__device__ float pow2_scale(float m) {
  if (!(m > 0.0f) || !(m <= 3.4028235e38f)) return 1.0f;
  int e = ilogbf(m) + 1 - 9;
  while (m > ldexpf(448.0f, e)) ++e;
  while (e > -126 && m <= ldexpf(448.0f, e - 1)) --e;
  return ldexpf(1.0f, e);
}

__global__ void k_fp8_finalize(const unsigned* __restrict__ amax, int n_layers, float* __restrict__ scales) {
  const int k = threadIdx.x;
  if (k < n_layers) {
    scales[2 * k] = pow2_scale(__uint_as_float(amax[k]));
    scales[2 * k + 1] = pow2_scale(__uint_as_float(amax[kMaxLayers + k]));
  }
}

// The weight-chunk table of the LDS kernel (offsets and lengths in 16-byte units: an FP8 operand is 8
// bytes, a 16-bit one 16, and every chunk holds a multiple of 64 operands) and its LDS size.
// staged: the LDS-staged BC epilogue (the heads reuse the chunk buffers, which must hold them).
// Bytes of the staging area at the start of the LDS: the two weight-chunk buffers, or the heads of
// the workgroup's waves (16 positions each) for the LDS-staged epilogue, whichever is larger.
size_t stage_bytes(int hid_inst, bool fp8, int head_stride, bool staged, int waves) {
  (void)fp8;  // FP8 mode's widest chunks are its bfloat16 layers: 16-byte operands like the 16-bit formats
  const size_t chunk = (size_t)kChunkTiles * (hid_inst / 16) * 64 * 16;
  const size_t ybytes = staged ? (size_t)waves * 16 * head_stride * sizeof(float) : 0;
  return std::max(2 * chunk, (ybytes + sizeof(u32x4) - 1) / sizeof(u32x4) * sizeof(u32x4));
}

int make_chunks(const Plan& p, bool fp8, int head_stride, bool staged, ChunkTable* ct, size_t* lds_out,
                int waves = kLdsWaves) {
  const Shape& s = p.s;
  const int64_t unit = fp8 ? 8 : 16;  // bytes of a pack_off unit
  *ct = ChunkTable{};
  for (int k = 0; k < s.n_layers; ++k) {
    // FP8 mode: E4M3 operands (8 bytes) in the middle layers, bfloat16 (16 bytes) in the first and the head
    const int64_t op_bytes = fp8 && k > 0 && k < s.n_layers - 1 ? 8 : 16;
    for (int t0 = 0; t0 < p.otiles[k]; t0 += kChunkTiles) {
      NTBC_REQUIRE(ct->n < kMaxChunks, "more than %d weight chunks", kMaxChunks);
      const int nt = std::min(kChunkTiles, p.otiles[k] - t0);
      ct->src[ct->n] = (p.pack_off[k] * unit + (int64_t)t0 * p.ksteps[k] * 64 * op_bytes) / 16;
      ct->len[ct->n] = (int)((int64_t)nt * p.ksteps[k] * 64 * op_bytes / 16);
      ++ct->n;
    }
  }
  int64_t nb = 0;
  for (int k = 0; k < s.n_layers; ++k) nb = std::max<int64_t>(nb, p.bias_off[k] + (int64_t)p.otiles[k] * 32);
  ct->n_bias = (int)((nb + 3) / 4 * 4);
  const size_t stage = stage_bytes(p.hid_inst, fp8, head_stride, staged, waves);
  ct->stage = (int)(stage / sizeof(u32x4));
  *lds_out = stage + (256 + (size_t)ct->n_bias) * sizeof(float);
  NTBC_REQUIRE(*lds_out <= 160 * 1024, "head_dim %d needs %zu bytes of LDS", s.head_dim, *lds_out);
  return NTBC_OK;
}

// The FP32 kernel's chunks: kF32ChunkTiles tiles of 16 rows over a layer's K-steps (4-byte operands).
int make_chunks_f32(const Plan& p, int head_stride, ChunkTable* ct, size_t* lds_out) {
  const Shape& s = p.s;
  *ct = ChunkTable{};
  for (int k = 0; k < s.n_layers; ++k) {
    for (int t0 = 0; t0 < p.otiles[k]; t0 += kF32ChunkTiles) {
      NTBC_REQUIRE(ct->n < kMaxChunks, "more than %d weight chunks", kMaxChunks);
      const int nt = std::min(kF32ChunkTiles, p.otiles[k] - t0);
      ct->src[ct->n] = (p.pack_off[k] + (int64_t)t0 * p.ksteps[k] * 64) * 4 / 16;
      ct->len[ct->n] = (int)((int64_t)nt * p.ksteps[k] * 64 * 4 / 16);
      ++ct->n;
    }
  }
  int64_t nb = 0;
  for (int k = 0; k < s.n_layers; ++k) nb = std::max<int64_t>(nb, p.bias_off[k] + (int64_t)p.otiles[k] * 16);
  ct->n_bias = (int)((nb + 3) / 4 * 4);
  const size_t chunk = (size_t)kF32ChunkTiles * (p.hid_inst / 4) * 64 * 4;
  const size_t ybytes = (size_t)kF32Waves * 16 * head_stride * sizeof(float);
  const size_t stage = std::max(2 * chunk, (ybytes + sizeof(u32x4) - 1) / sizeof(u32x4) * sizeof(u32x4));
  ct->stage = (int)(stage / sizeof(u32x4));
  *lds_out = stage + (256 + (size_t)ct->n_bias) * sizeof(float);
  NTBC_REQUIRE(*lds_out <= 160 * 1024, "head_dim %d needs %zu bytes of LDS", s.head_dim, *lds_out);
  return NTBC_OK;
}

}  // namespace

// ------------------------------------------------------------------------------ kernel instances
// The fused 16-bit/FP8 kernels exist per (precision, hidden width, first-layer K-steps, unrolled
// middle layers, register-epilogue texture mix); the host code finds one through these lookups, each
// defined in the part that compiles its instances.
namespace ntbc {
typedef void (*LdsLaunch)(dim3, dim3, size_t, hipStream_t, const void* args, const void* chunks);
typedef void (*BatchLaunch)(dim3, dim3, size_t, hipStream_t, const void* items, int n_items, unsigned* done,
                            uint64_t* stamps);
bool lds_instance_bf16(int hid, int ks0, int nh, int nb1, int nb4, const void** fn, LdsLaunch* launch);
bool lds_instance_fp16(int hid, int ks0, int nh, int nb1, int nb4, const void** fn, LdsLaunch* launch);
bool lds_instance_fp8(int hid, int ks0, int nh, int nb1, int nb4, const void** fn, LdsLaunch* launch);
bool batch_instance_bf16(int hid, int ks0, int nh, int nb1, int nb4, int waves, const void** fn, BatchLaunch* launch);
bool batch_instance_fp16(int hid, int ks0, int nh, int nb1, int nb4, int waves, const void** fn, BatchLaunch* launch);
bool batch_instance_fp8(int hid, int ks0, int nh, int nb1, int nb4, int waves, const void** fn, BatchLaunch* launch);
bool lds_instance_f32(int hid, int kq, const void** fn, LdsLaunch* launch);
}  // namespace ntbc

// Single-range instances: every precision at widths 64/128/256 with one to four input K-steps and a
// run-time layer count, the two-middle-layer shapes (128, 3) and (256, 4) unrolled, with the LDS-staged
// epilogue and with the register epilogue for two BC1 + three BC4 textures.
#define NTBC_LDS_INSTANCE_L(LP, H, K, NH, NB1, NB4)                                                          \
  if (hid == H && ks0 == K && nh == NH && nb1 == NB1 && (NB1 < 0 || nb4 == NB4)) {                         \
    *fn = (const void*)k_infer_lds<LP, H, K, NH, NB1, NB4>;                                                  \
    *launch = [](dim3 gr, dim3 bl, size_t sh, hipStream_t st, const void* x, const void* y) {               \
      hipLaunchKernelGGL((k_infer_lds<LP, H, K, NH, NB1, NB4>), gr, bl, sh, st,                             \
                         *static_cast<const InferArgs*>(x), *static_cast<const ChunkTable*>(y));            \
    };                                                                                                       \
    return true;                                                                                             \
  }
#define NTBC_LDS_INSTANCES(LP)                                                                                    \
  NTBC_LDS_INSTANCE_L(LP, 64, 1, -1, -1, 0) NTBC_LDS_INSTANCE_L(LP, 64, 2, -1, -1, 0)                            \
  NTBC_LDS_INSTANCE_L(LP, 64, 3, -1, -1, 0) NTBC_LDS_INSTANCE_L(LP, 64, 4, -1, -1, 0)                            \
  NTBC_LDS_INSTANCE_L(LP, 128, 1, -1, -1, 0) NTBC_LDS_INSTANCE_L(LP, 128, 2, -1, -1, 0)                          \
  NTBC_LDS_INSTANCE_L(LP, 128, 3, -1, -1, 0) NTBC_LDS_INSTANCE_L(LP, 128, 4, -1, -1, 0)                          \
  NTBC_LDS_INSTANCE_L(LP, 256, 1, -1, -1, 0) NTBC_LDS_INSTANCE_L(LP, 256, 2, -1, -1, 0)                          \
  NTBC_LDS_INSTANCE_L(LP, 256, 3, -1, -1, 0) NTBC_LDS_INSTANCE_L(LP, 256, 4, -1, -1, 0)                          \
  NTBC_LDS_INSTANCE_L(LP, 128, 3, 2, -1, 0) NTBC_LDS_INSTANCE_L(LP, 256, 4, 2, -1, 0)                            \
  NTBC_LDS_INSTANCE_L(LP, 128, 3, 2, 2, 3) NTBC_LDS_INSTANCE_L(LP, 256, 4, 2, 2, 3)

// Batched instances: the same shapes with the LDS-staged epilogue in every precision, and BF16 with the
// register epilogue for two BC1 + one to three BC4 textures at widths 64, 128 (run-time layer count)
// and 256 (two middle layers unrolled).
#define NTBC_BATCH_INSTANCE_L(LP, H, K, NH, NB1, NB4)                                                         \
  if (hid == H && ks0 == K && nh == NH && nb1 == NB1 && (NB1 < 0 || nb4 == NB4) && waves == NTBC_BATCH_W) {   \
    *fn = (const void*)k_infer_lds_batch<LP, H, K, NH, NB1, NB4, NTBC_BATCH_W>;                              \
    *launch = [](dim3 g, dim3 b, size_t sh, hipStream_t st, const void* it, int n, unsigned* d, uint64_t* s) { \
      hipLaunchKernelGGL((k_infer_lds_batch<LP, H, K, NH, NB1, NB4, NTBC_BATCH_W>), g, b, sh, st,           \
                         static_cast<const BatchItem*>(it), n, d, s);                                        \
    };                                                                                                       \
    return true;                                                                                             \
  }
#define NTBC_BATCH_INSTANCES(LP)                                                                                    \
  NTBC_BATCH_INSTANCE_L(LP, 64, 1, -1, -1, 0) NTBC_BATCH_INSTANCE_L(LP, 64, 2, -1, -1, 0)                          \
  NTBC_BATCH_INSTANCE_L(LP, 64, 3, -1, -1, 0) NTBC_BATCH_INSTANCE_L(LP, 64, 4, -1, -1, 0)                          \
  NTBC_BATCH_INSTANCE_L(LP, 128, 1, -1, -1, 0) NTBC_BATCH_INSTANCE_L(LP, 128, 2, -1, -1, 0)                        \
  NTBC_BATCH_INSTANCE_L(LP, 128, 3, -1, -1, 0) NTBC_BATCH_INSTANCE_L(LP, 128, 4, -1, -1, 0)                        \
  NTBC_BATCH_INSTANCE_L(LP, 256, 1, -1, -1, 0) NTBC_BATCH_INSTANCE_L(LP, 256, 2, -1, -1, 0)                        \
  NTBC_BATCH_INSTANCE_L(LP, 256, 3, -1, -1, 0) NTBC_BATCH_INSTANCE_L(LP, 256, 4, -1, -1, 0)                        \
  NTBC_BATCH_INSTANCE_L(LP, 128, 3, 2, -1, 0) NTBC_BATCH_INSTANCE_L(LP, 256, 4, 2, -1, 0)
#define NTBC_BATCH_REG(H, K, NH)                                                                                \
  NTBC_BATCH_INSTANCE_L(Lp::BF16, H, K, NH, 2, 1) NTBC_BATCH_INSTANCE_L(Lp::BF16, H, K, NH, 2, 2)                 \
  NTBC_BATCH_INSTANCE_L(Lp::BF16, H, K, NH, 2, 3)

namespace ntbc {
#if NTBC_PART(1)
bool lds_instance_bf16(int hid, int ks0, int nh, int nb1, int nb4, const void** fn, LdsLaunch* launch) {
  NTBC_LDS_INSTANCES(Lp::BF16)
  return false;
}
#endif
#if NTBC_PART(2)
bool lds_instance_fp16(int hid, int ks0, int nh, int nb1, int nb4, const void** fn, LdsLaunch* launch) {
  NTBC_LDS_INSTANCES(Lp::FP16)
  return false;
}
#endif
#if NTBC_PART(3)
bool lds_instance_fp8(int hid, int ks0, int nh, int nb1, int nb4, const void** fn, LdsLaunch* launch) {
  NTBC_LDS_INSTANCES(Lp::FP8)
  return false;
}
#endif
// BF16 batched instances come in three tile shapes (2, 4 or 8 waves of 32 positions per workgroup),
// one per part, for the tile autotuner; FP16 and FP8 in the default shape (4 waves).
#define NTBC_BATCH_BF16_W(WV)                                                                                   \
  bool batch_instance_bf16_w##WV(int hid, int ks0, int nh, int nb1, int nb4, int waves, const void** fn,         \
                                 BatchLaunch* launch) {                                                         \
    NTBC_BATCH_INSTANCES(Lp::BF16)                                                                              \
    NTBC_BATCH_REG(64, 4, -1) NTBC_BATCH_REG(128, 4, -1) NTBC_BATCH_REG(256, 4, 2)                              \
    return false;                                                                                               \
  }
bool batch_instance_bf16_w2(int, int, int, int, int, int, const void**, BatchLaunch*);
bool batch_instance_bf16_w4(int, int, int, int, int, int, const void**, BatchLaunch*);
bool batch_instance_bf16_w8(int, int, int, int, int, int, const void**, BatchLaunch*);
#if NTBC_PART(4)
#define NTBC_BATCH_W 4
NTBC_BATCH_BF16_W(4)
#undef NTBC_BATCH_W
bool batch_instance_bf16(int hid, int ks0, int nh, int nb1, int nb4, int waves, const void** fn, BatchLaunch* launch) {
  if (waves == 2) return batch_instance_bf16_w2(hid, ks0, nh, nb1, nb4, waves, fn, launch);
  if (waves == 8) return batch_instance_bf16_w8(hid, ks0, nh, nb1, nb4, waves, fn, launch);
  return batch_instance_bf16_w4(hid, ks0, nh, nb1, nb4, waves, fn, launch);
}
#endif
#if NTBC_PART(7)
#define NTBC_BATCH_W 2
NTBC_BATCH_BF16_W(2)
#undef NTBC_BATCH_W
#endif
#if NTBC_PART(8)
#define NTBC_BATCH_W 8
NTBC_BATCH_BF16_W(8)
#undef NTBC_BATCH_W
#endif
#define NTBC_BATCH_W 4
#if NTBC_PART(5)
bool batch_instance_fp16(int hid, int ks0, int nh, int nb1, int nb4, int waves, const void** fn, BatchLaunch* launch) {
  NTBC_BATCH_INSTANCES(Lp::FP16)
  return false;
}
#endif
#if NTBC_PART(6)
bool batch_instance_fp8(int hid, int ks0, int nh, int nb1, int nb4, int waves, const void** fn, BatchLaunch* launch) {
  NTBC_BATCH_INSTANCES(Lp::FP8)
  return false;
}
#endif
#undef NTBC_BATCH_W
#undef NTBC_BATCH_BF16_W
#if NTBC_PART(10)
// FP32 LDS-staged instances: widths 64/128/256, one to four groups of 16 first-layer inputs.
#define NTBC_F32_INSTANCE(H, KQ)                                                                        \
  if (hid == H && kq == KQ) {                                                                           \
    *fn = (const void*)k_infer_f32_lds<H, KQ>;                                                          \
    *launch = [](dim3 gr, dim3 bl, size_t sh, hipStream_t st, const void* x, const void* y) {          \
      hipLaunchKernelGGL((k_infer_f32_lds<H, KQ>), gr, bl, sh, st, *static_cast<const InferArgs*>(x), \
                         *static_cast<const ChunkTable*>(y));                                           \
    };                                                                                                  \
    return true;                                                                                        \
  }
bool lds_instance_f32(int hid, int kq, const void** fn, LdsLaunch* launch) {
  NTBC_F32_INSTANCE(64, 1) NTBC_F32_INSTANCE(64, 2) NTBC_F32_INSTANCE(64, 3) NTBC_F32_INSTANCE(64, 4)
  NTBC_F32_INSTANCE(128, 1) NTBC_F32_INSTANCE(128, 2) NTBC_F32_INSTANCE(128, 3) NTBC_F32_INSTANCE(128, 4)
  NTBC_F32_INSTANCE(256, 1) NTBC_F32_INSTANCE(256, 2) NTBC_F32_INSTANCE(256, 3) NTBC_F32_INSTANCE(256, 4)
  return false;
}
#undef NTBC_F32_INSTANCE
#endif
}  // namespace ntbc
#undef NTBC_LDS_INSTANCE_L
#undef NTBC_LDS_INSTANCES
#undef NTBC_BATCH_INSTANCE_L
#undef NTBC_BATCH_INSTANCES
#undef NTBC_BATCH_REG

// ------------------------------------------------------------------------------ host code (part 0)
#if NTBC_PART(0)
namespace {

struct BatchGroup {
  int32_t lp, hid, ks0, nh, nb1, nb4;
  int32_t item_begin, item_end;
  int64_t tiles, lds;
  int32_t waves;       // tile shape: waves (of 32 block positions) per workgroup
  int32_t pad;
  int64_t lds_w[3];    // LDS bytes at 2, 4 and 8 waves
};

constexpr int kTileWaves[3] = {2, 4, 8};
int waves_index(int w) { return w == 2 ? 0 : (w == 8 ? 2 : 1); }

// Kernel instance of an item: the unrolled two-middle-layer instances where they exist, else the
// generic one (same selection as ntbc_infer_blocks).
int batch_nh(const Plan& p) {
  const int mid = p.s.n_layers - 2;
  const bool special = (p.hid_inst == 256 && p.ksteps[0] == 4) || (p.hid_inst == 128 && p.ksteps[0] == 3);
  return special && mid == 2 ? 2 : -1;
}

int launch_batch_group(const BatchGroup& gr, const BatchItem* items, unsigned* done, uint64_t* stamps, hipStream_t strm) {
  const void* fn = nullptr;
  BatchLaunch launch = nullptr;
  const bool found =
      gr.lp == NTBC_FP8_E4M3 ? batch_instance_fp8(gr.hid, gr.ks0, gr.nh, gr.nb1, gr.nb4, gr.waves, &fn, &launch)
      : gr.lp == NTBC_FP16   ? batch_instance_fp16(gr.hid, gr.ks0, gr.nh, gr.nb1, gr.nb4, gr.waves, &fn, &launch)
                             : batch_instance_bf16(gr.hid, gr.ks0, gr.nh, gr.nb1, gr.nb4, gr.waves, &fn, &launch);
  if (!found) fn = nullptr;
  NTBC_REQUIRE(fn != nullptr, "no batch kernel instance for width %d, %d input K-steps, %d-wave tiles", gr.hid, gr.ks0,
               gr.waves);
  NTBC_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)gr.lds));
  launch(dim3((unsigned)gr.tiles), dim3(64 * gr.waves), (size_t)gr.lds, strm, items + gr.item_begin,
         gr.item_end - gr.item_begin, done, stamps);
  return check_launch("ntbc_infer_batch");
}

// Register-resident BC epilogue (see RegLayout): the slot layout of a model when the fused kernel has
// an instance for its texture mix and network shape, else nb1 = -1 (heads staged in LDS).
struct RegPlan {
  int nb1 = -1, nb4 = 0;
  int tex[NTBC_MAX_TEXTURES] = {};
};

// Instances with the register epilogue: single range (any precision) for two BC1 + three BC4 textures
// at the paper-scale and 1024^2 shapes; batched (BF16) for two BC1 + one to three BC4 textures at
// widths 64, 128 (four input K-steps, run-time layer count) and 256 (four K-steps, two middle layers).
bool reg_instance(const Plan& p, int nb1, int nb4, bool batch) {
  if (batch) {
    const bool shape = (p.hid_inst == 256 && p.ksteps[0] == 4 && batch_nh(p) == 2) ||
                       ((p.hid_inst == 64 || p.hid_inst == 128) && p.ksteps[0] == 4 && batch_nh(p) == -1);
    return p.precision == NTBC_BF16 && shape && nb1 == 2 && nb4 >= 1 && nb4 <= 3;
  }
  const bool shape = (p.hid_inst == 256 && p.ksteps[0] == 4) || (p.hid_inst == 128 && p.ksteps[0] == 3);
  return shape && batch_nh(p) == 2 && nb1 == 2 && nb4 == 3;
}

RegPlan reg_plan(const Plan& p, bool batch = false) {
  const Shape& s = p.s;
  RegPlan r;
  int nb1 = 0, nb4 = 0;
  for (int t = 0; t < s.n_textures; ++t)
    if (s.formats[t] == NTBC_BC1) r.tex[nb1++] = t;
  for (int t = 0; t < s.n_textures; ++t)
    if (s.formats[t] == NTBC_BC4) r.tex[nb1 + nb4++] = t;
  if (!s.naive && reg_instance(p, nb1, nb4, batch) && 27 * nb1 + 9 * nb4 <= 16 * p.otiles[s.n_layers - 1]) {
    r.nb1 = nb1;
    r.nb4 = nb4;
  }
  return r;
}

// Canonical head neuron of packed head row `row` under the register layout, -1 for a padding row.
int reg_source(const Shape& s, const RegPlan& r, int row) {
  const int t = row / 32, q = (row % 32) / 8, g = (row % 8) / 4, slot = 16 * t + 4 * q + row % 4;
  const int c4 = 24 * r.nb1, e1 = c4 + 8 * r.nb4, e4 = e1 + 3 * r.nb1, used = e4 + r.nb4;
  if (slot < c4)
    return s.endpoint_dim + (8 * g + (slot % 24) / 3) * s.channels + s.ch_off[r.tex[slot / 24]] + slot % 3;
  if (slot < e1) return s.endpoint_dim + (8 * g + (slot - c4) % 8) * s.channels + s.ch_off[r.tex[r.nb1 + (slot - c4) / 8]];
  if (slot < e4) return s.ep_off[r.tex[(slot - e1) / 3]] + 3 * g + (slot - e1) % 3;
  if (slot < used) return s.ep_off[r.tex[r.nb1 + slot - e4]] + g;
  return -1;
}

void apply_reg_plan(const Shape& s, const RegPlan& r, PackArgs* pa, InferArgs* a) {
  if (r.nb1 < 0) return;
  if (pa) {
    pa->head_perm = 1;
    for (int row = 0; row < kHeadRows; ++row) pa->head_src[row] = (int16_t)reg_source(s, r, row);
  }
  if (!a) return;
  for (int k = 0; k < r.nb1 + r.nb4; ++k) {
    a->reg_tex[k] = r.tex[k];
    a->reg_ep[k] = s.ep_off[r.tex[k]];
    a->reg_ch[k] = s.ch_off[r.tex[k]];
  }
}

// Kernel arguments common to inference and calibration: the grid view, the packed-weight plan and the
// texture layout (block range, outputs and workspace pointers are set by the caller).
InferArgs infer_args(const Plan& p, const ntbc_model_desc* d, const ntbc_params* prm) {
  const Shape& s = p.s;
  InferArgs a{};
  a.grid.u8 = d->grid_dtype == NTBC_GRID_U8 ? static_cast<const uint8_t*>(prm->grid) : nullptr;
  a.grid.f32 = d->grid_dtype == NTBC_GRID_F32 ? static_cast<const float*>(prm->grid) : nullptr;
  a.grid.scale = prm->grid_scale;
  a.grid.zero = prm->grid_zero;
  a.grid.n_levels = s.n_levels;
  a.grid.base_res = s.base_res;
  a.grid.n_features = s.n_features;
  a.grid.blocks_w = s.blocks_w;
  a.grid.blocks_h = s.blocks_h;
  for (int l = 0; l <= s.n_levels; ++l) a.grid.level_offset[l] = s.level_offset[l];
  a.grid.shift_x = pow2_shift(s, s.blocks_w);
  a.grid.shift_y = pow2_shift(s, s.blocks_h);
  a.grid.fast8 = a.grid.u8 != nullptr && s.n_features == 8 && a.grid.shift_x >= 0 && a.grid.shift_y >= 0 &&
                 s.level_offset[s.n_levels] * 8 < (1ll << 31);
  for (int k = 0; k < s.n_layers; ++k) {
    a.pack_off[k] = p.pack_off[k];
    a.bias_off[k] = p.bias_off[k];
    a.ksteps[k] = p.ksteps[k];
    a.otiles[k] = p.otiles[k];
  }
  a.n_layers = s.n_layers;
  a.head_dim = s.head_dim;
  a.head_stride = s.head_dim | 1;
  a.n_textures = s.n_textures;
  for (int t = 0; t < s.n_textures; ++t) {
    a.formats[t] = s.formats[t];
    a.ep_off[t] = s.ep_off[t];
    a.ch_off[t] = s.ch_off[t];
  }
  a.endpoint_dim = s.endpoint_dim;
  a.channels = s.channels;
  a.naive = s.naive;
  a.fp8_scales = prm->fp8_scales;
  a.stride = 1;
  return a;
}

}  // namespace

extern "C" int ntbc_workspace_size(const ntbc_model_desc* d, int32_t precision, int64_t batch, size_t* bytes) {
  NTBC_REQUIRE(bytes != nullptr, "bytes is NULL");
  NTBC_REQUIRE(batch >= 0, "batch %lld < 0", (long long)batch);
  if (batch > 0) {
    Shape s;
    int st = make_shape(d, &s);
    if (st != NTBC_OK) return st;
    int64_t need = train_workspace_bytes(s, batch);
    Plan p;
    if (make_plan(d, precision, &p) == NTBC_OK && p.total_bytes > need) need = p.total_bytes;
    *bytes = (size_t)need;
    return NTBC_OK;
  }
  Plan p;
  int st = make_plan(d, precision, &p);
  if (st != NTBC_OK) return st;
  *bytes = (size_t)p.total_bytes;
  return NTBC_OK;
}

namespace {

// ntbc_infer_blocks with the workspace already chosen (the caller's buffer, or the device's static
// scratch array for ntbc_infer_blocks_noalloc); `p` is the plan of (d, precision).
int infer_blocks(const Plan& p, const ntbc_model_desc* d, const ntbc_params* prm, int32_t precision,
                 int64_t first_block, int64_t n_blocks, uint64_t* blocks_out, float* heads_out, void* workspace,
                 size_t workspace_bytes, void* stream) {
  int st = NTBC_OK;
  const Shape& s = p.s;
  NTBC_REQUIRE(prm != nullptr && prm->grid != nullptr && prm->weights != nullptr, "params, grid or weights is NULL");
  if (d->grid_dtype == NTBC_GRID_U8)
    NTBC_REQUIRE(prm->grid_scale != nullptr && prm->grid_zero != nullptr, "U8 grid needs grid_scale and grid_zero");
  NTBC_REQUIRE(first_block >= 0 && n_blocks >= 0 && first_block + n_blocks <= s.n_positions,
               "block range [%lld, %lld) outside 0..%lld", (long long)first_block,
               (long long)(first_block + n_blocks), (long long)s.n_positions);
  const bool lp16 = precision == NTBC_BF16 || precision == NTBC_FP16;
  const bool fp8 = precision == NTBC_FP8_E4M3;
  const bool lds_shape = p.otiles[s.n_layers - 1] <= kHeadTiles && p.ksteps[0] <= 4 && s.n_layers >= 2;
  if (fp8) {
    NTBC_REQUIRE(prm->fp8_scales != nullptr, "FP8 needs fp8_scales (see ntbc_fp8_calibrate)");
    if (!lds_shape || s.n_layers < 3)
      return fail(NTBC_EUNSUPPORTED, "FP8 needs head_dim <= %d, in_dim <= 64 and two hidden layers", 32 * kHeadTiles);
  }
  if (n_blocks == 0) return NTBC_OK;
  NTBC_REQUIRE(blocks_out != nullptr, "blocks_out is NULL");
  if (workspace == nullptr || workspace_bytes < (size_t)p.total_bytes)
    return fail(NTBC_ENOWORKSPACE, "workspace needs %lld bytes", (long long)p.total_bytes);
  hipStream_t strm = as_stream(stream);

  char* ws = static_cast<char*>(workspace);
  void* wpack = ws;
  float* bias = reinterpret_cast<float*>(ws + ((p.pack_bytes + 255) / 256) * 256);

  PackArgs pa{};
  pa.w = prm->weights;
  pa.n_layers = s.n_layers;
  for (int k = 0; k < s.n_layers; ++k) {
    pa.in_dim[k] = s.layer_in[k];
    pa.out_dim[k] = s.layer_out[k];
    pa.w_off[k] = s.w_off[k];
    pa.b_off[k] = s.b_off[k];
    pa.ksteps[k] = p.ksteps[k];
    pa.otiles[k] = p.otiles[k];
    pa.pack_off[k] = p.pack_off[k];
    pa.bias_off[k] = p.bias_off[k];
  }
  pa.fp8_scales = prm->fp8_scales;
  InferArgs a = infer_args(p, d, prm);
  const RegPlan rp = (lp16 || fp8) && lds_shape ? reg_plan(p) : RegPlan{};
  apply_reg_plan(s, rp, &pa, &a);
  if (!(prm->flags & NTBC_REUSE_PACKED)) {
    const dim3 pgrid(64, s.n_layers);
    if (fp8)
      hipLaunchKernelGGL(k_pack_lp<Lp::FP8>, pgrid, dim3(256), 0, strm, pa, static_cast<u32x2*>(wpack), bias);
    else if (precision == NTBC_BF16)
      hipLaunchKernelGGL(k_pack_lp<Lp::BF16>, pgrid, dim3(256), 0, strm, pa, static_cast<u32x4*>(wpack), bias);
    else if (precision == NTBC_FP16)
      hipLaunchKernelGGL(k_pack_lp<Lp::FP16>, pgrid, dim3(256), 0, strm, pa, static_cast<u32x4*>(wpack), bias);
    else
      hipLaunchKernelGGL(k_pack_f32, pgrid, dim3(256), 0, strm, pa, static_cast<float*>(wpack), bias);
    st = check_launch("ntbc_infer_blocks: weight packing");
    if (st != NTBC_OK) return st;
  }

  a.wpack = wpack;
  a.bias = bias;
  a.first = first_block;
  a.n = n_blocks;
  a.out = blocks_out;
  a.heads = heads_out;

  const int ppw = p.positions_per_wave;
  if ((lp16 || fp8) && lds_shape) {
    ChunkTable ct{};
    size_t lds = 0;
    st = make_chunks(p, fp8, a.head_stride, rp.nb1 < 0, &ct, &lds);
    if (st != NTBC_OK) return st;
    const int64_t nwg = ceil_div(n_blocks, (int64_t)32 * kLdsWaves);
    const void* fn = nullptr;
    LdsLaunch launch = nullptr;
    const int nh = batch_nh(p);
    const bool found = fp8 ? lds_instance_fp8(p.hid_inst, p.ksteps[0], nh, rp.nb1, rp.nb4, &fn, &launch)
                       : precision == NTBC_FP16 ? lds_instance_fp16(p.hid_inst, p.ksteps[0], nh, rp.nb1, rp.nb4, &fn, &launch)
                                                : lds_instance_bf16(p.hid_inst, p.ksteps[0], nh, rp.nb1, rp.nb4, &fn, &launch);
    if (!found) fn = nullptr;
    NTBC_REQUIRE(fn != nullptr, "no LDS kernel instance for width %d, %d input K-steps", p.hid_inst, p.ksteps[0]);
    NTBC_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    launch(dim3((unsigned)nwg), dim3(64 * kLdsWaves), lds, strm, &a, &ct);
    return check_launch("ntbc_infer_blocks");
  }
  if (precision == NTBC_FP32 && p.otiles[s.n_layers - 1] <= kF32HeadTiles && p.ksteps[0] <= 16 && s.n_layers >= 2) {
    ChunkTable ct{};
    size_t lds = 0;
    st = make_chunks_f32(p, a.head_stride, &ct, &lds);
    if (st != NTBC_OK) return st;
    const void* fn = nullptr;
    LdsLaunch launch = nullptr;
    if (!lds_instance_f32(p.hid_inst, p.ksteps[0] / 4, &fn, &launch)) fn = nullptr;
    NTBC_REQUIRE(fn != nullptr, "no FP32 kernel instance for width %d, %d input K-steps", p.hid_inst, p.ksteps[0]);
    NTBC_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    launch(dim3((unsigned)ceil_div(n_blocks, (int64_t)16 * kF32Waves)), dim3(64 * kF32Waves), lds, strm, &a, &ct);
    return check_launch("ntbc_infer_blocks");
  }
  const int64_t nwg = ceil_div(n_blocks, (int64_t)ppw * kWaves);
  const size_t lds = (size_t)kWaves * ppw * a.head_stride * sizeof(float);
  const dim3 grid((unsigned)nwg), block(64 * kWaves);
  NTBC_REQUIRE(lds <= 160 * 1024, "head_dim %d needs %zu bytes of LDS", s.head_dim, lds);
  if (lds > 64 * 1024) {
    const void* fn = precision == NTBC_BF16
                         ? (p.hid_inst == 64 ? (const void*)k_infer_lp<Lp::BF16, 64>
                                             : (p.hid_inst == 128 ? (const void*)k_infer_lp<Lp::BF16, 128>
                                                                  : (const void*)k_infer_lp<Lp::BF16, 256>))
                     : precision == NTBC_FP16
                         ? (p.hid_inst == 64 ? (const void*)k_infer_lp<Lp::FP16, 64>
                                             : (p.hid_inst == 128 ? (const void*)k_infer_lp<Lp::FP16, 128>
                                                                  : (const void*)k_infer_lp<Lp::FP16, 256>))
                         : (p.hid_inst == 64 ? (const void*)k_infer_f32<64, false>
                                             : (p.hid_inst == 128 ? (const void*)k_infer_f32<128, false> : (const void*)k_infer_f32<256, false>));
    NTBC_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  }
  if (precision == NTBC_BF16) {
    if (p.hid_inst == 64) hipLaunchKernelGGL((k_infer_lp<Lp::BF16, 64>), grid, block, lds, strm, a);
    else if (p.hid_inst == 128) hipLaunchKernelGGL((k_infer_lp<Lp::BF16, 128>), grid, block, lds, strm, a);
    else hipLaunchKernelGGL((k_infer_lp<Lp::BF16, 256>), grid, block, lds, strm, a);
  } else if (precision == NTBC_FP16) {
    if (p.hid_inst == 64) hipLaunchKernelGGL((k_infer_lp<Lp::FP16, 64>), grid, block, lds, strm, a);
    else if (p.hid_inst == 128) hipLaunchKernelGGL((k_infer_lp<Lp::FP16, 128>), grid, block, lds, strm, a);
    else hipLaunchKernelGGL((k_infer_lp<Lp::FP16, 256>), grid, block, lds, strm, a);
  } else {
    if (p.hid_inst == 64) hipLaunchKernelGGL((k_infer_f32<64, false>), grid, block, lds, strm, a);
    else if (p.hid_inst == 128) hipLaunchKernelGGL((k_infer_f32<128, false>), grid, block, lds, strm, a);
    else hipLaunchKernelGGL((k_infer_f32<256, false>), grid, block, lds, strm, a);
  }
  return check_launch("ntbc_infer_blocks");
}

// Per-device scratch of ntbc_infer_blocks_noalloc: the packed weights and biases live here instead of
// in a caller workspace.  Each GPU holds its own copy of the array until the process ends.
constexpr size_t kScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device id, set on first use

// The device address of the current device's copy of `scratch` (the array's name is only a host-side
// stand-in); looked up once per device.
int scratch_address(void** out) {
  int dev = -1;
  NTBC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(NTBC_EUNSUPPORTED, "device %d beyond %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return fail(NTBC_EHIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return NTBC_OK;
}

}  // namespace

extern "C" int ntbc_infer_blocks(const ntbc_model_desc* d, const ntbc_params* prm, int32_t precision,
                                 int64_t first_block, int64_t n_blocks, uint64_t* blocks_out, float* heads_out,
                                 void* workspace, size_t workspace_bytes, void* stream) {
  Plan p;
  int st = make_plan(d, precision, &p);
  if (st != NTBC_OK) return st;
  return infer_blocks(p, d, prm, precision, first_block, n_blocks, blocks_out, heads_out, workspace,
                      workspace_bytes, stream);
}

extern "C" int ntbc_infer_blocks_noalloc(const ntbc_model_desc* d, const ntbc_params* prm, int32_t precision,
                                         int64_t first_block, int64_t n_blocks, uint64_t* blocks_out,
                                         float* heads_out, void* stream) {
  Plan p;
  int st = make_plan(d, precision, &p);
  if (st != NTBC_OK) return st;
  if ((size_t)p.total_bytes > kScratchBytes)
    return fail(NTBC_ENOWORKSPACE, "model needs %lld bytes of packed weights, beyond the %zu-byte static scratch",
                (long long)p.total_bytes, kScratchBytes);
  void* ws = nullptr;
  st = scratch_address(&ws);
  if (st != NTBC_OK) return st;
  return infer_blocks(p, d, prm, precision, first_block, n_blocks, blocks_out, heads_out, ws, kScratchBytes, stream);
}

extern "C" int ntbc_fp8_calibrate(const ntbc_model_desc* d, const ntbc_params* prm, int64_t n_sample, float* scales_out,
                                  void* workspace, size_t workspace_bytes, void* stream) {
  Plan p8, p;
  int st = make_plan(d, NTBC_FP8_E4M3, &p8);
  if (st != NTBC_OK) return st;
  st = make_plan(d, NTBC_FP32, &p);
  if (st != NTBC_OK) return st;
  const Shape& s = p.s;
  NTBC_REQUIRE(prm != nullptr && prm->grid != nullptr && prm->weights != nullptr, "params, grid or weights is NULL");
  if (d->grid_dtype == NTBC_GRID_U8)
    NTBC_REQUIRE(prm->grid_scale != nullptr && prm->grid_zero != nullptr, "U8 grid needs grid_scale and grid_zero");
  NTBC_REQUIRE(n_sample >= 1, "n_sample %lld < 1", (long long)n_sample);
  NTBC_REQUIRE(scales_out != nullptr, "scales_out is NULL");
  if (workspace == nullptr || workspace_bytes < (size_t)p8.total_bytes)
    return fail(NTBC_ENOWORKSPACE, "workspace needs %lld bytes", (long long)p8.total_bytes);
  hipStream_t strm = as_stream(stream);

  char* ws = static_cast<char*>(workspace) + p8.calib_offset;
  float* wpack = reinterpret_cast<float*>(ws);
  float* bias = reinterpret_cast<float*>(ws + ((p.pack_bytes + 255) / 256) * 256);
  unsigned* amax = reinterpret_cast<unsigned*>(ws + p.total_bytes);  // 2 * kMaxLayers words
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, strm, amax, 2 * kMaxLayers);

  PackArgs pa{};
  pa.w = prm->weights;
  pa.n_layers = s.n_layers;
  WMaxArgs wm{};
  wm.w = prm->weights;
  wm.n_layers = s.n_layers;
  wm.amax = amax;
  for (int k = 0; k < s.n_layers; ++k) {
    pa.in_dim[k] = s.layer_in[k];
    pa.out_dim[k] = s.layer_out[k];
    pa.w_off[k] = s.w_off[k];
    pa.b_off[k] = s.b_off[k];
    pa.ksteps[k] = p.ksteps[k];
    pa.otiles[k] = p.otiles[k];
    pa.pack_off[k] = p.pack_off[k];
    pa.bias_off[k] = p.bias_off[k];
    wm.w_off[k] = s.w_off[k];
    wm.count[k] = (int64_t)s.layer_in[k] * s.layer_out[k];
  }
  hipLaunchKernelGGL(k_pack_f32, dim3(64, s.n_layers), dim3(256), 0, strm, pa, wpack, bias);
  hipLaunchKernelGGL(k_weight_absmax, dim3(64, s.n_layers), dim3(256), 0, strm, wm);
  st = check_launch("ntbc_fp8_calibrate: weights");
  if (st != NTBC_OK) return st;

  InferArgs a = infer_args(p, d, prm);
  a.wpack = wpack;
  a.bias = bias;
  a.first = 0;
  a.n = std::min<int64_t>(n_sample, s.n_positions);
  a.stride = std::max<int64_t>(1, s.n_positions / n_sample);
  a.amax = amax;
  const dim3 grid((unsigned)ceil_div(a.n, (int64_t)16 * kWaves)), block(64 * kWaves);
  if (p.hid_inst == 64) hipLaunchKernelGGL((k_infer_f32<64, true>), grid, block, 0, strm, a);
  else if (p.hid_inst == 128) hipLaunchKernelGGL((k_infer_f32<128, true>), grid, block, 0, strm, a);
  else hipLaunchKernelGGL((k_infer_f32<256, true>), grid, block, 0, strm, a);
  st = check_launch("ntbc_fp8_calibrate: activations");
  if (st != NTBC_OK) return st;
  hipLaunchKernelGGL(k_fp8_finalize, dim3(1), dim3(64), 0, strm, amax, s.n_layers, scales_out);
  return check_launch("ntbc_fp8_calibrate");
}

// ------------------------------------------------------------------------------ batched decode, host
namespace {

constexpr int32_t kBatchMagic = 0x4E544243;
constexpr int kMaxBatchGroups = 32;

struct BatchPack {
  PackArgs pa;
  void* pack;
  float* bias;
};

struct BatchHeader {
  int32_t magic, n_items, n_groups, n_packs, precision, pad;
  int64_t workspace_bytes, done_offset, packs_offset, items_offset;
  BatchGroup groups[kMaxBatchGroups];
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t batch_table_bytes(int n) {
  return align_up(sizeof(BatchHeader), 16) + align_up((size_t)n * sizeof(BatchPack), 16) + (size_t)n * sizeof(BatchItem);
}

const BatchHeader* batch_header(const void* table) {
  const BatchHeader* h = static_cast<const BatchHeader*>(table);
  return h != nullptr && h->magic == kBatchMagic ? h : nullptr;
}

}  // namespace

extern "C" int ntbc_batch_table_size(int32_t n_items, size_t* bytes) {
  NTBC_REQUIRE(n_items >= 1 && bytes != nullptr, "n_items %d < 1 or bytes is NULL", n_items);
  *bytes = batch_table_bytes(n_items);
  return NTBC_OK;
}

extern "C" int ntbc_batch_plan(const ntbc_batch_item* items, int32_t n_items, int32_t precision, void* workspace,
                               void* table, size_t table_bytes, size_t* workspace_bytes) {
  NTBC_REQUIRE(items != nullptr && n_items >= 1, "items is NULL or n_items %d < 1", n_items);
  NTBC_REQUIRE(table != nullptr && table_bytes >= batch_table_bytes(n_items), "table is NULL or smaller than %zu bytes",
               batch_table_bytes(n_items));
  NTBC_REQUIRE(workspace_bytes != nullptr, "workspace_bytes is NULL");
  NTBC_REQUIRE(precision == NTBC_BF16 || precision == NTBC_FP16 || precision == NTBC_FP8_E4M3,
               "batched decode runs in BF16, FP16 or FP8 (precision %d)", precision);
  std::vector<Plan> plans(n_items);
  std::vector<int> model_of(n_items), key(n_items);
  std::vector<int32_t> model_ids;
  std::vector<int64_t> model_off;
  std::vector<int> model_item;
  std::vector<BatchGroup> groups;
  int64_t off = 0;
  for (int i = 0; i < n_items; ++i) {
    const ntbc_batch_item& it = items[i];
    int st = make_plan(&it.desc, precision, &plans[i]);
    if (st != NTBC_OK) return st;
    const Plan& p = plans[i];
    const Shape& s = p.s;
    NTBC_REQUIRE(it.params.grid != nullptr && it.params.weights != nullptr, "item %d: grid or weights is NULL", i);
    if (it.desc.grid_dtype == NTBC_GRID_U8)
      NTBC_REQUIRE(it.params.grid_scale != nullptr && it.params.grid_zero != nullptr, "item %d: U8 grid needs scale and zero", i);
    if (precision == NTBC_FP8_E4M3) NTBC_REQUIRE(it.params.fp8_scales != nullptr, "item %d: FP8 needs fp8_scales", i);
    NTBC_REQUIRE(it.first_block >= 0 && it.n_blocks >= 0 && it.first_block + it.n_blocks <= s.n_positions,
                 "item %d: block range outside the block grid", i);
    NTBC_REQUIRE(it.n_blocks == 0 || it.blocks_out != nullptr, "item %d: blocks_out is NULL", i);
    if (!(p.otiles[s.n_layers - 1] <= kHeadTiles && p.ksteps[0] <= 4 && s.n_layers >= 2))
      return fail(NTBC_EUNSUPPORTED, "item %d: batched decode needs head_dim <= %d, in_dim <= 64 and a hidden layer", i,
                  32 * kHeadTiles);
    if (precision == NTBC_FP8_E4M3 && s.n_layers < 3)
      return fail(NTBC_EUNSUPPORTED, "item %d: FP8 needs two hidden layers", i);
    int m = -1;
    for (size_t q = 0; q < model_ids.size(); ++q)
      if (model_ids[q] == it.model_id) m = (int)q;
    if (m < 0) {
      m = (int)model_ids.size();
      model_ids.push_back(it.model_id);
      model_item.push_back(i);
      model_off.push_back(off);
      off = (int64_t)align_up((size_t)(off + p.total_bytes), 256);
    } else {
      const Plan& q = plans[model_item[m]];
      bool same = q.s.n_layers == s.n_layers && q.total_bytes == p.total_bytes && q.s.n_textures == s.n_textures;
      for (int k = 0; same && k < s.n_layers; ++k) same = q.s.layer_in[k] == s.layer_in[k] && q.s.layer_out[k] == s.layer_out[k];
      for (int t = 0; same && t < s.n_textures; ++t) same = q.s.formats[t] == s.formats[t];
      NTBC_REQUIRE(same && items[model_item[m]].params.weights == it.params.weights,
                   "item %d: model_id %d shared by items with different weights, layer shapes or textures", i, it.model_id);
    }
    model_of[i] = m;
    const RegPlan rp = reg_plan(p, true);
    const BatchGroup want{precision, p.hid_inst, p.ksteps[0], batch_nh(p), rp.nb1, rp.nb4, 0, 0, 0, 0, kLdsWaves, 0, {0, 0, 0}};
    int gi = -1;
    for (size_t q = 0; q < groups.size(); ++q)
      if (groups[q].hid == want.hid && groups[q].ks0 == want.ks0 && groups[q].nh == want.nh &&
          groups[q].nb1 == want.nb1 && groups[q].nb4 == want.nb4)
        gi = (int)q;
    if (gi < 0) {
      NTBC_REQUIRE((int)groups.size() < kMaxBatchGroups, "more than %d kernel instances in one batch", kMaxBatchGroups);
      gi = (int)groups.size();
      groups.push_back(want);
    }
    key[i] = gi;
  }
  const int64_t done_offset = off;
  const int64_t need = (int64_t)align_up((size_t)(done_offset + 4 * (int64_t)n_items), 256);
  *workspace_bytes = (size_t)need;

  char* base = static_cast<char*>(table);
  BatchHeader* h = reinterpret_cast<BatchHeader*>(base);
  *h = BatchHeader{};
  h->magic = kBatchMagic;
  h->n_items = n_items;
  h->precision = precision;
  h->workspace_bytes = need;
  h->done_offset = done_offset;
  h->packs_offset = (int64_t)align_up(sizeof(BatchHeader), 16);
  h->items_offset = h->packs_offset + (int64_t)align_up((size_t)n_items * sizeof(BatchPack), 16);
  BatchPack* packs = reinterpret_cast<BatchPack*>(base + h->packs_offset);
  BatchItem* out = reinterpret_cast<BatchItem*>(base + h->items_offset);
  char* ws = static_cast<char*>(workspace);
  for (size_t m = 0; m < model_ids.size(); ++m) {
    const int i = model_item[m];
    const Plan& p = plans[i];
    const Shape& s = p.s;
    BatchPack bp{};
    bp.pa.w = items[i].params.weights;
    bp.pa.n_layers = s.n_layers;
    for (int k = 0; k < s.n_layers; ++k) {
      bp.pa.in_dim[k] = s.layer_in[k];
      bp.pa.out_dim[k] = s.layer_out[k];
      bp.pa.w_off[k] = s.w_off[k];
      bp.pa.b_off[k] = s.b_off[k];
      bp.pa.ksteps[k] = p.ksteps[k];
      bp.pa.otiles[k] = p.otiles[k];
      bp.pa.pack_off[k] = p.pack_off[k];
      bp.pa.bias_off[k] = p.bias_off[k];
    }
    bp.pa.fp8_scales = items[i].params.fp8_scales;
    apply_reg_plan(s, reg_plan(p, true), &bp.pa, nullptr);  // head rows permuted for the register epilogue
    bp.pack = ws ? ws + model_off[m] : nullptr;
    bp.bias = ws ? reinterpret_cast<float*>(ws + model_off[m] + (int64_t)align_up((size_t)p.pack_bytes, 256)) : nullptr;
    packs[m] = bp;
  }
  h->n_packs = (int)model_ids.size();
  int n_out = 0;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    BatchGroup& gr = groups[gi];
    gr.item_begin = n_out;
    int64_t tiles = 0;
    for (int i = 0; i < n_items; ++i) {
      if (key[i] != (int)gi || items[i].n_blocks == 0) continue;
      const Plan& p = plans[i];
      BatchItem bi{};
      bi.a = infer_args(p, &items[i].desc, &items[i].params);
      apply_reg_plan(p.s, reg_plan(p, true), nullptr, &bi.a);
      bi.a.wpack = packs[model_of[i]].pack;
      bi.a.bias = packs[model_of[i]].bias;
      bi.a.first = items[i].first_block;
      bi.a.n = items[i].n_blocks;
      bi.a.out = items[i].blocks_out;
      bi.a.heads = nullptr;
      const bool fp8 = precision == NTBC_FP8_E4M3, staged = reg_plan(p, true).nb1 < 0;
      size_t lds = 0;
      int st = make_chunks(p, fp8, bi.a.head_stride, staged, &bi.ct, &lds, gr.waves);
      if (st != NTBC_OK) return st;
      // LDS of every tile shape (the staging area grows with the waves of the staged epilogue)
      for (int w = 0; w < 3; ++w) {
        const int64_t lw = (int64_t)stage_bytes(p.hid_inst, fp8, bi.a.head_stride, staged, kTileWaves[w]) +
                           (256 + (int64_t)bi.ct.n_bias) * (int64_t)sizeof(float);
        gr.lds_w[w] = std::max<int64_t>(gr.lds_w[w], lw);
      }
      gr.lds = gr.lds_w[waves_index(gr.waves)];
      bi.tile_begin = tiles;
      bi.tiles = ceil_div(items[i].n_blocks, (int64_t)32 * gr.waves);
      bi.index = i;
      tiles += bi.tiles;
      out[n_out++] = bi;
    }
    gr.item_end = n_out;
    gr.tiles = tiles;
  }
  h->n_groups = (int)groups.size();
  for (size_t gi = 0; gi < groups.size(); ++gi) h->groups[gi] = groups[gi];
  return NTBC_OK;
}

extern "C" int ntbc_batch_pack(const void* table, void* workspace, size_t workspace_bytes, void* stream) {
  const BatchHeader* h = batch_header(table);
  NTBC_REQUIRE(h != nullptr, "table is not a batch plan");
  NTBC_REQUIRE(workspace != nullptr && workspace_bytes >= (size_t)h->workspace_bytes,
               "workspace needs %lld bytes", (long long)h->workspace_bytes);
  hipStream_t strm = as_stream(stream);
  const BatchPack* packs = reinterpret_cast<const BatchPack*>(static_cast<const char*>(table) + h->packs_offset);
  for (int m = 0; m < h->n_packs; ++m) {
    const BatchPack& bp = packs[m];
    NTBC_REQUIRE(bp.pack != nullptr, "the plan was made without a workspace");
    const dim3 pgrid(64, bp.pa.n_layers);
    if (h->precision == NTBC_FP8_E4M3)
      hipLaunchKernelGGL(k_pack_lp<Lp::FP8>, pgrid, dim3(256), 0, strm, bp.pa, static_cast<u32x2*>(bp.pack), bp.bias);
    else if (h->precision == NTBC_FP16)
      hipLaunchKernelGGL(k_pack_lp<Lp::FP16>, pgrid, dim3(256), 0, strm, bp.pa, static_cast<u32x4*>(bp.pack), bp.bias);
    else
      hipLaunchKernelGGL(k_pack_lp<Lp::BF16>, pgrid, dim3(256), 0, strm, bp.pa, static_cast<u32x4*>(bp.pack), bp.bias);
    int st = check_launch("ntbc_batch_pack");
    if (st != NTBC_OK) return st;
  }
  return NTBC_OK;
}

extern "C" int ntbc_batch_groups(const void* table, int32_t* groups_out, int32_t max_groups, int32_t* n_groups) {
  const BatchHeader* h = batch_header(table);
  NTBC_REQUIRE(h != nullptr, "table is not a batch plan");
  NTBC_REQUIRE(n_groups != nullptr, "n_groups is NULL");
  *n_groups = h->n_groups;
  for (int g = 0; g < h->n_groups && g < max_groups && groups_out != nullptr; ++g) {
    const BatchGroup& gr = h->groups[g];
    const int32_t row[8] = {gr.lp, gr.hid, gr.ks0, gr.nh, gr.nb1, gr.nb4, gr.waves, gr.item_end - gr.item_begin};
    for (int k = 0; k < 8; ++k) groups_out[8 * g + k] = row[k];
  }
  return NTBC_OK;
}

extern "C" int ntbc_batch_set_waves(void* table, int32_t group, int32_t waves) {
  BatchHeader* h = const_cast<BatchHeader*>(batch_header(table));
  NTBC_REQUIRE(h != nullptr, "table is not a batch plan");
  NTBC_REQUIRE(group >= 0 && group < h->n_groups, "group %d outside 0..%d", group, h->n_groups - 1);
  NTBC_REQUIRE(waves == 2 || waves == 4 || waves == 8, "waves %d is not 2, 4 or 8", waves);
  BatchGroup& gr = h->groups[group];
  if (gr.lp != NTBC_BF16 && waves != kLdsWaves)
    return fail(NTBC_EUNSUPPORTED, "only the BF16 batch has %d-wave tiles", waves);
  const int64_t lds = gr.lds_w[waves_index(waves)];
  NTBC_REQUIRE(lds <= 160 * 1024, "%d-wave tiles of group %d need %lld bytes of LDS", waves, group, (long long)lds);
  gr.waves = waves;
  gr.lds = lds;
  BatchItem* items = reinterpret_cast<BatchItem*>(static_cast<char*>(table) + h->items_offset);
  int64_t tiles = 0;
  for (int i = gr.item_begin; i < gr.item_end; ++i) {
    // the staging area (and with it the /255 table and biases behind it) moves with the shape
    items[i].ct.stage = (int)(stage_bytes(gr.hid, gr.lp == NTBC_FP8_E4M3, items[i].a.head_stride, gr.nb1 < 0, waves) /
                              sizeof(u32x4));
    items[i].tile_begin = tiles;
    items[i].tiles = ceil_div(items[i].a.n, (int64_t)32 * waves);
    tiles += items[i].tiles;
  }
  gr.tiles = tiles;
  return NTBC_OK;
}

extern "C" int ntbc_infer_batch(const void* table, const void* table_device, void* workspace, size_t workspace_bytes,
                                uint64_t* stamps, void* stream) {
  const BatchHeader* h = batch_header(table);
  NTBC_REQUIRE(h != nullptr, "table is not a batch plan");
  NTBC_REQUIRE(table_device != nullptr, "table_device is NULL");
  NTBC_REQUIRE(workspace != nullptr && workspace_bytes >= (size_t)h->workspace_bytes,
               "workspace needs %lld bytes", (long long)h->workspace_bytes);
  hipStream_t strm = as_stream(stream);
  unsigned* done = reinterpret_cast<unsigned*>(static_cast<char*>(workspace) + h->done_offset);
  hipLaunchKernelGGL(k_batch_start, dim3(1), dim3(256), 0, strm, done, h->n_items, stamps);
  int st = check_launch("ntbc_infer_batch: start");
  if (st != NTBC_OK) return st;
  const BatchItem* items = reinterpret_cast<const BatchItem*>(static_cast<const char*>(table_device) + h->items_offset);
  for (int gi = 0; gi < h->n_groups; ++gi) {
    if (h->groups[gi].tiles == 0) continue;
    st = launch_batch_group(h->groups[gi], items, done, stamps, strm);
    if (st != NTBC_OK) return st;
  }
  return NTBC_OK;
}
#endif  // NTBC_PART(0)

// ------------------------------------------------------------------------------ the paper's own layout
// One model of the paper's network layout (Sec. 3.4): an endpoint network on the block's grid cell and
// a colour network on each of its 16 texels' cells, each 2 features per grid level (at most 16
// inputs: one K-step), three hidden layers of 64 SELU units and sigmoid outputs, with half-precision
// operands and float32 accumulation.  A wave owns 32 blocks: one endpoint-network run and 16
// colour-network runs (texel i of the 32 blocks at a time), all with the layers chained in registers
// as in the kernels above; the sigmoid outputs go to LDS in the NTBC head layout and the LDS-staged BC
// epilogue packs them (Eq. dist), exactly as for the one-trunk model.
#if NTBC_PART(9)
namespace {

constexpr int kFaWaves = 2;                    // waves (of 32 blocks) per workgroup
constexpr int kFaHidden = 64;
constexpr int kFaLayers = 4;                   // three hidden layers and the head
constexpr float kSeluLambda = 1.0507009873554805f;
constexpr float kSeluLambdaAlpha = 1.0507009873554805f * 1.6732632423543772f;

struct FaNet {
  int64_t pack_off[kFaLayers];  // u32x4 units in the packed weights
  int bias_off[kFaLayers];      // floats in the padded biases
  int ksteps[kFaLayers];        // 1, 4, 4, 4
  int head_tiles;               // 32-row tiles of the outputs
  int n_out;
};

struct FaithArgs {
  InferArgs pk;                 // texture layout, block range, outputs, head stride (for pack_blocks)
  dev::GridView eg, cg;         // endpoint grid (cells = blocks), colour grid (cells = texels)
  const u32x4* wpack;
  const float* bias;
  FaNet ep, col;
};

__device__ __forceinline__ float selu(float z) {
  return z > 0.0f ? kSeluLambda * z : kSeluLambdaAlpha * (__expf(z) - 1.0f);
}

// SELU of a hidden tile's accumulators (started from the biases) -> the next layer's two B operands.
__device__ __forceinline__ void selu_epilogue(const f32x16_t& acc, u32x4* lo, u32x4* hi) {
  float r[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) r[v] = selu(acc[v]);
  *lo = x8_of<Lp::FP16>(r);
  *hi = x8_of<Lp::FP16>(r + 8);
}

// One network run on the 32 positions of the wave (layer-0 operand x0): the first n.n_out sigmoid
// outputs of position j go to y[j * hs + col0 + k].
__device__ __forceinline__ void fa_net(const FaithArgs& a, const FaNet& n, const u32x4& x0, float* y, int hs, int col0,
                                       int lane) {
  const int j = lane & 31, g = lane >> 5;
  // the weights and biases are re-read from the cache on every run (opaque base pointers keep the
  // compiler from hoisting all of them into registers across the 17 runs, which would leave one wave
  // per SIMD)
  const u32x4* wp = a.wpack;
  const float* bias = a.bias;
  asm volatile("" : "+s"(wp), "+s"(bias));
  u32x4 h[4], o[4];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    f32x16_t acc = acc_init<Lp::FP16>(bias + n.bias_off[0] + 32 * t, g);
    acc = mfma16<Lp::FP16>(wp[n.pack_off[0] + (int64_t)t * 64 + lane], x0, acc);
    selu_epilogue(acc, &h[2 * t], &h[2 * t + 1]);
  }
#pragma unroll
  for (int l = 1; l < kFaLayers - 1; ++l) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      f32x16_t acc = acc_init<Lp::FP16>(bias + n.bias_off[l] + 32 * t, g);
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = mfma16<Lp::FP16>(wp[n.pack_off[l] + ((int64_t)t * 4 + s) * 64 + lane], h[s], acc);
      selu_epilogue(acc, &o[2 * t], &o[2 * t + 1]);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) h[s] = o[s];
  }
  for (int t = 0; t < n.head_tiles; ++t) {
    f32x16_t acc = acc_init<Lp::FP16>(bias + n.bias_off[kFaLayers - 1] + 32 * t, g);
#pragma unroll
    for (int s = 0; s < 4; ++s)
      acc = mfma16<Lp::FP16>(wp[n.pack_off[kFaLayers - 1] + ((int64_t)t * 4 + s) * 64 + lane], h[s], acc);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int neuron = 32 * t + 8 * (v / 4) + 4 * g + (v % 4);
      if (neuron < n.n_out) y[j * hs + col0 + neuron] = sigmoid(acc[v]);
    }
  }
}

// Colour-grid gather of a texel split in two so that the loads of the next texel are in flight while
// the current texel's network runs: the corner loads (uint8 grid, 2 features a vertex: one 16-bit load
// per corner) and bilinear weights of the lane's four levels (features 8g .. 8g+7), then the blend.
struct FaTaps {
  uint32_t raw[4][4];
  float w[4][4];
};

__device__ __forceinline__ void fa_load_u8(const dev::GridView& g, int gi, int tx, int ty, FaTaps& t) {
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int level = 4 * gi + h;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      t.raw[h][c] = 0;
      t.w[h][c] = 0.0f;
    }
    if (level < g.n_levels) {
      const int res = g.base_res << level;
      const dev::Corner cx = g.shift_x >= 0 ? dev::corner_pow2(tx, g.blocks_w, res, g.shift_x) : dev::corner(tx, g.blocks_w, res);
      const dev::Corner cy = g.shift_y >= 0 ? dev::corner_pow2(ty, g.blocks_h, res, g.shift_y) : dev::corner(ty, g.blocks_h, res);
      const int64_t v00 = g.level_offset[level] + (int64_t)cy.i0 * res + cx.i0;
      const uint16_t* p = reinterpret_cast<const uint16_t*>(g.u8);
      t.raw[h][0] = p[v00];
      t.raw[h][1] = p[v00 + 1];
      t.raw[h][2] = p[v00 + res];
      t.raw[h][3] = p[v00 + res + 1];
      t.w[h][0] = (1.0f - cx.f) * (1.0f - cy.f);
      t.w[h][1] = cx.f * (1.0f - cy.f);
      t.w[h][2] = (1.0f - cx.f) * cy.f;
      t.w[h][3] = cx.f * cy.f;
    }
  }
}

__device__ __forceinline__ void fa_blend_u8(const dev::GridView& g, int gi, const FaTaps& t, float v[8]) {
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int level = 4 * gi + h;
    const bool on = level < g.n_levels;
    const float s = on ? g.scale[level] : 0.0f;
    const float sz = on ? -s * (float)g.zero[level] : 0.0f;
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      float q[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) q[c] = (float)((t.raw[h][c] >> (8 * f)) & 255u);
      v[2 * h + f] = on ? fmaf(s, fmaf(t.w[h][0], q[0], fmaf(t.w[h][1], q[1], fmaf(t.w[h][2], q[2], t.w[h][3] * q[3]))), sz)
                        : 0.0f;
    }
  }
}

__global__ void __launch_bounds__(64 * kFaWaves) k_faithful(FaithArgs a) {
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 31, g = lane >> 5;
  const int64_t pos0 = a.pk.first + ((int64_t)blockIdx.x * kFaWaves + wave) * 32;
  const int64_t last = a.pk.first + a.pk.n - 1;
  const int64_t id = pos0 + j <= last ? pos0 + j : last;
  const int bx = (int)(id % a.eg.blocks_w), by = (int)(id / a.eg.blocks_w);
  const int hs = a.pk.head_stride;
  float* y = lds + wave * 32 * hs;
  float v[8];
  dev::features<8>(a.eg, 8 * g, bx, by, v);
  fa_net(a, a.ep, x8_of<Lp::FP16>(v), y, hs, 0, lane);
  if (a.cg.u8) {
    // texel i + 1's corner loads are issued before texel i's network runs
    FaTaps taps;
    fa_load_u8(a.cg, g, 4 * bx, 4 * by, taps);
#pragma unroll 1
    for (int i = 0; i < 16; ++i) {
      fa_blend_u8(a.cg, g, taps, v);
      const u32x4 x = x8_of<Lp::FP16>(v);
      if (i < 15) fa_load_u8(a.cg, g, 4 * bx + ((i + 1) & 3), 4 * by + ((i + 1) >> 2), taps);
      fa_net(a, a.col, x, y, hs, a.pk.endpoint_dim + i * a.pk.channels, lane);
    }
  } else {
#pragma unroll 1
    for (int i = 0; i < 16; ++i) {
      dev::features<8>(a.cg, 8 * g, 4 * bx + (i & 3), 4 * by + (i >> 2), v);
      fa_net(a, a.col, x8_of<Lp::FP16>(v), y, hs, a.pk.endpoint_dim + i * a.pk.channels, lane);
    }
  }
  __syncthreads();
  // inlined here: an out-of-line call would take the kernel argument by address, i.e. copy it to scratch
  [[clang::always_inline]] pack_blocks<32>(a.pk, y, lane, pos0);
}

// Shape of one model of the paper's layout.
struct FaShape {
  int E, C, in_ep, in_col, ep_tiles;
  int64_t n_ep, n_col;                  // canonical FP32 weights of each network
  int64_t pack_units, bias_floats;      // packed operands (u32x4) and padded biases of both networks
  FaNet ep, col;
  PackArgs pa_ep, pa_col;
};

int64_t fa_net_weights(int in, int out) {
  return (int64_t)in * kFaHidden + kFaHidden + 2 * ((int64_t)kFaHidden * kFaHidden + kFaHidden) + (int64_t)kFaHidden * out + out;
}

void fa_plan_net(int in, int out, int64_t* units, int64_t* bias, FaNet* n, PackArgs* pa) {
  const int dims[kFaLayers + 1] = {in, kFaHidden, kFaHidden, kFaHidden, out};
  *pa = PackArgs{};
  pa->n_layers = kFaLayers;
  int64_t w = 0;
  n->n_out = out;
  n->head_tiles = (out + 31) / 32;
  for (int k = 0; k < kFaLayers; ++k) {
    pa->in_dim[k] = dims[k];
    pa->out_dim[k] = dims[k + 1];
    pa->w_off[k] = w;
    w += (int64_t)dims[k] * dims[k + 1];
    pa->b_off[k] = w;
    w += dims[k + 1];
    n->ksteps[k] = k == 0 ? 1 : 4;
    pa->ksteps[k] = n->ksteps[k];
    pa->otiles[k] = k == kFaLayers - 1 ? n->head_tiles : 2;
    pa->pack_off[k] = *units;
    n->pack_off[k] = *units;
    *units += (int64_t)pa->otiles[k] * pa->ksteps[k] * 64;
    pa->bias_off[k] = *bias;
    n->bias_off[k] = (int)*bias;
    *bias += 32 * pa->otiles[k];
  }
}

int fa_shape(const ntbc_faithful_desc* d, FaShape* s) {
  NTBC_REQUIRE(d != nullptr, "desc is NULL");
  NTBC_REQUIRE(d->ep_levels >= 1 && d->ep_levels <= 8 && d->col_levels >= 1 && d->col_levels <= 8,
               "grid levels (%d, %d) must be 1..8 (2 features each: at most 16 inputs)", d->ep_levels, d->col_levels);
  NTBC_REQUIRE(d->ep_base_res >= 2 && d->col_base_res >= 2, "base resolutions must be >= 2");
  NTBC_REQUIRE(((int64_t)d->ep_base_res << (d->ep_levels - 1)) <= 32768 &&
                   ((int64_t)d->col_base_res << (d->col_levels - 1)) <= 32768,
               "finest grid level too large");
  NTBC_REQUIRE(d->grid_dtype == NTBC_GRID_F32 || d->grid_dtype == NTBC_GRID_U8, "bad grid_dtype %d", d->grid_dtype);
  NTBC_REQUIRE(d->n_textures >= 1 && d->n_textures <= NTBC_MAX_TEXTURES, "n_textures %d out of range", d->n_textures);
  NTBC_REQUIRE(d->blocks_w >= 1 && d->blocks_h >= 1 && (int64_t)d->blocks_w * 4 <= 65536 && (int64_t)d->blocks_h * 4 <= 65536,
               "block grid %dx%d out of range", d->blocks_w, d->blocks_h);
  *s = FaShape{};
  for (int t = 0; t < d->n_textures; ++t) {
    NTBC_REQUIRE(d->formats[t] == NTBC_BC1 || d->formats[t] == NTBC_BC4, "formats[%d] = %d", t, d->formats[t]);
    s->E += d->formats[t] == NTBC_BC1 ? 6 : 2;
    s->C += d->formats[t] == NTBC_BC1 ? 3 : 1;
  }
  NTBC_REQUIRE(s->E <= 64 && s->C <= 32, "endpoint outputs %d > 64 or colour outputs %d > 32", s->E, s->C);
  s->in_ep = 2 * d->ep_levels;
  s->in_col = 2 * d->col_levels;
  s->n_ep = fa_net_weights(s->in_ep, s->E);
  s->n_col = fa_net_weights(s->in_col, s->C);
  fa_plan_net(s->in_ep, s->E, &s->pack_units, &s->bias_floats, &s->ep, &s->pa_ep);
  fa_plan_net(s->in_col, s->C, &s->pack_units, &s->bias_floats, &s->col, &s->pa_col);
  s->ep_tiles = s->ep.head_tiles;
  return NTBC_OK;
}

size_t fa_workspace(const FaShape& s) { return (size_t)s.pack_units * 16 + 256 + (size_t)s.bias_floats * 4; }

dev::GridView fa_grid(int levels, int base, int blocks_w, int blocks_h, int u8, const void* grid, const float* scale,
                      const int32_t* zero) {
  Shape sh{};
  sh.n_levels = levels;
  sh.base_res = base;
  dev::GridView g{};
  g.u8 = u8 ? static_cast<const uint8_t*>(grid) : nullptr;
  g.f32 = u8 ? nullptr : static_cast<const float*>(grid);
  g.scale = scale;
  g.zero = zero;
  g.n_levels = levels;
  g.base_res = base;
  g.n_features = 2;
  g.blocks_w = blocks_w;
  g.blocks_h = blocks_h;
  int64_t off = 0;
  for (int l = 0; l < levels; ++l) {
    g.level_offset[l] = off;
    off += ((int64_t)base << l) * ((int64_t)base << l);
  }
  g.level_offset[levels] = off;
  g.shift_x = pow2_shift(sh, blocks_w);
  g.shift_y = pow2_shift(sh, blocks_h);
  g.fast8 = 0;
  return g;
}

}  // namespace

extern "C" int ntbc_faithful_sizes(const ntbc_faithful_desc* d, int64_t* ep_weights, int64_t* col_weights,
                                   size_t* workspace_bytes) {
  FaShape s;
  int st = fa_shape(d, &s);
  if (st != NTBC_OK) return st;
  if (ep_weights) *ep_weights = s.n_ep;
  if (col_weights) *col_weights = s.n_col;
  if (workspace_bytes) *workspace_bytes = fa_workspace(s);
  return NTBC_OK;
}

extern "C" int ntbc_faithful_infer(const ntbc_faithful_desc* d, const ntbc_faithful_params* p, int64_t first_block,
                                   int64_t n_blocks, uint64_t* blocks_out, float* heads_out, void* workspace,
                                   size_t workspace_bytes, void* stream) {
  FaShape s;
  int st = fa_shape(d, &s);
  if (st != NTBC_OK) return st;
  NTBC_REQUIRE(p != nullptr && p->ep_grid && p->col_grid && p->ep_weights && p->col_weights, "params: a NULL pointer");
  NTBC_REQUIRE(d->grid_dtype != NTBC_GRID_U8 || (p->ep_scale && p->ep_zero && p->col_scale && p->col_zero),
               "params: U8 grids need their scales and zero points");
  const int64_t npos = (int64_t)d->blocks_w * d->blocks_h;
  NTBC_REQUIRE(first_block >= 0 && n_blocks >= 0 && first_block + n_blocks <= npos, "block range out of the grid");
  if (n_blocks == 0) return NTBC_OK;
  NTBC_REQUIRE(blocks_out != nullptr, "blocks_out is NULL");
  if (workspace == nullptr || workspace_bytes < fa_workspace(s))
    return fail(NTBC_ENOWORKSPACE, "workspace needs %zu bytes", fa_workspace(s));
  hipStream_t strm = as_stream(stream);
  u32x4* pack = static_cast<u32x4*>(workspace);
  float* bias = reinterpret_cast<float*>(static_cast<char*>(workspace) + (size_t)s.pack_units * 16 + 256);
  // both networks' FP16 operands (layer 0 in input order, the hidden layers in the chained order)
  s.pa_ep.w = p->ep_weights;
  s.pa_col.w = p->col_weights;
  hipLaunchKernelGGL(k_pack_lp<Lp::FP16>, dim3(64, kFaLayers), dim3(256), 0, strm, s.pa_ep, pack, bias);
  hipLaunchKernelGGL(k_pack_lp<Lp::FP16>, dim3(64, kFaLayers), dim3(256), 0, strm, s.pa_col, pack, bias);
  st = check_launch("ntbc_faithful_infer: pack");
  if (st != NTBC_OK) return st;
  FaithArgs a{};
  InferArgs& k = a.pk;
  k.n_textures = d->n_textures;
  int e = 0, c = 0;
  for (int t = 0; t < d->n_textures; ++t) {
    k.formats[t] = d->formats[t];
    k.ep_off[t] = e;
    k.ch_off[t] = c;
    e += d->formats[t] == NTBC_BC1 ? 6 : 2;
    c += d->formats[t] == NTBC_BC1 ? 3 : 1;
  }
  k.endpoint_dim = s.E;
  k.channels = s.C;
  k.head_dim = s.E + 16 * s.C;
  k.head_stride = k.head_dim | 1;
  k.first = first_block;
  k.n = n_blocks;
  k.out = blocks_out;
  k.heads = heads_out;
  const int u8 = d->grid_dtype == NTBC_GRID_U8;
  a.eg = fa_grid(d->ep_levels, d->ep_base_res, d->blocks_w, d->blocks_h, u8, p->ep_grid, p->ep_scale, p->ep_zero);
  a.cg = fa_grid(d->col_levels, d->col_base_res, 4 * d->blocks_w, 4 * d->blocks_h, u8, p->col_grid, p->col_scale,
                 p->col_zero);
  a.wpack = pack;
  a.bias = bias;
  a.ep = s.ep;
  a.col = s.col;
  const size_t lds = (size_t)kFaWaves * 32 * k.head_stride * sizeof(float);
  NTBC_REQUIRE(lds <= 160 * 1024, "heads need %zu bytes of LDS", lds);
  NTBC_HIP(hipFuncSetAttribute((const void*)k_faithful, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const unsigned blocks = (unsigned)ceil_div(n_blocks, 32 * kFaWaves);
  hipLaunchKernelGGL(k_faithful, dim3(blocks), dim3(64 * kFaWaves), lds, strm, a);
  return check_launch("k_faithful");
}
#endif  // NTBC_PART(9)
