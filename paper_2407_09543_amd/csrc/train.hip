// NTBC training on gfx950 (paper Sec. 3.2 training procedure, Sec. 3.3 grid QAT, Sec. 3.4 optimiser,
// App. A straight-through estimator).  One step for a batch of block positions:
//
//   k_level_minmax / k_qat_params   per-level min/max of the FP32 master grid -> (s_l, z_l) (QAT on)
//   k_features                      bilinear features of the (fake-quantised) grid -> X [B][in]
//   k_gemm (bias+ReLU / sigmoid)    MLP forward, every layer's input kept for the batch
//   k_loss_grad                     L_e, L_c and both decoded-colour terms, dL/dY with the STE
//   k_dsigmoid                      dZ_out = dY * Y (1 - Y) (in the training step: inside k_loss_grad)
//   k_gemm (mask / split-K atomic)  dH_k = dZ_k W_k masked by ReLU, dW_k = dZ_k^T H_k, db by k_colsum
//                                   (bfloat16 products: db fused into the dW product)
//   k_scatter                       dX through the bilinear weights into d_grid (atomic), QAT
//                                   pass-through mask
//   k_adam                          dense bias-corrected Adam, learning rate from the host schedule
//
// The autograd entry points (ntbc_forward / ntbc_backward) keep nothing between calls: the backward
// pass recomputes the forward activations of its batch.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "common.h"
#include "device.h"

namespace {

using namespace ntbc;

constexpr int kBlock = 256;

// ------------------------------------------------------------------------------------------ layout
struct TrainLayout {
  // float offsets into the workspace
  int64_t stats;  // [4][NTBC_MAX_LEVELS]: min (ordered int), max (ordered int), s (float), z (int)
  int64_t x, h[4], y, dy, da, db;
  int64_t total;
};

TrainLayout train_layout(const Shape& s, int64_t batch) {
  TrainLayout t{};
  int64_t o = 0;
  auto take = [&](int64_t n) {
    const int64_t r = o;
    o += (n + 63) / 64 * 64;
    return r;
  };
  t.stats = take(4 * NTBC_MAX_LEVELS);
  t.x = take(batch * s.in_dim);
  for (int k = 0; k < s.n_hidden; ++k) t.h[k] = take(batch * s.hidden);
  t.y = take(batch * s.head_dim);
  t.dy = take(batch * s.head_dim);
  const int w = s.hidden > s.in_dim ? s.hidden : s.in_dim;
  t.da = take(batch * w);
  t.db = take(batch * w);
  t.total = o;
  return t;
}

// ------------------------------------------------------------------------------------------ helpers
// p[0 .. n) = v: 16-byte non-temporal stores over the 16-byte aligned body (the zeroed gradient is not
// read before the scatter's atomics, and the stores then do not evict what the kernels between read),
// single stores for the (< 4) floats before and after it.
__global__ void k_fill(float* __restrict__ p, int64_t n, float v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t head = std::min<int64_t>(n, (int64_t)(((16 - (reinterpret_cast<uintptr_t>(p) & 15)) & 15) / 4));
  const int64_t n4 = (n - head) / 4, done = head + 4 * n4;
  if (t < head) p[t] = v;
  typedef float f4 __attribute__((ext_vector_type(4)));
  f4* q = reinterpret_cast<f4*>(p + head);
  for (int64_t i = t; i < n4; i += stride) __builtin_nontemporal_store(f4{v, v, v, v}, q + i);
  if (t < n - done) p[done + t] = v;
}

__device__ __forceinline__ int ordered(float f) {
  const int i = __float_as_int(f);
  return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__device__ __forceinline__ float unordered(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7FFFFFFF); }

__global__ void k_init_stats(int* __restrict__ stats) {
  const int l = threadIdx.x;
  if (l < NTBC_MAX_LEVELS) {
    stats[l] = 0x7FFFFFFF;
    stats[NTBC_MAX_LEVELS + l] = (int)0x80000000;
  }
}

struct LevelArgs {
  int n_levels;
  int64_t begin[NTBC_MAX_LEVELS], count[NTBC_MAX_LEVELS];  // in floats
};

// Per-level min/max of the master grid.  Block b handles a contiguous slice of one level (blocks are
// assigned to levels in proportion to their sizes by the host); the block reduces in LDS and issues
// one atomic pair.
struct MinMaxArgs {
  const float* g;
  int n_levels;
  int64_t begin[NTBC_MAX_LEVELS], count[NTBC_MAX_LEVELS];
  int first_block[NTBC_MAX_LEVELS + 1];  // blocks [first_block[l], first_block[l+1]) cover level l
};

__global__ void __launch_bounds__(kBlock) k_level_minmax(MinMaxArgs a, int* __restrict__ stats) {
  __shared__ int smin[kBlock / 64], smax[kBlock / 64];
  int l = 0;
  while (l + 1 < a.n_levels && (int)blockIdx.x >= a.first_block[l + 1]) ++l;
  const int nb = a.first_block[l + 1] - a.first_block[l];
  const int b = blockIdx.x - a.first_block[l];
  const int64_t n = a.count[l];
  const int64_t per = (n + nb - 1) / nb;
  const int64_t i0 = (int64_t)b * per, i1 = min(n, i0 + per);
  const float* p = a.g + a.begin[l];
  int mn = 0x7FFFFFFF, mx = (int)0x80000000;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
    const int o = ordered(p[i]);
    mn = min(mn, o);
    mx = max(mx, o);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mn = min(mn, __shfl_xor(mn, off));
    mx = max(mx, __shfl_xor(mx, off));
  }
  if ((threadIdx.x & 63) == 0) {
    smin[threadIdx.x >> 6] = mn;
    smax[threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) {
      mn = min(mn, smin[w]);
      mx = max(mx, smax[w]);
    }
    atomicMin(&stats[l], mn);
    atomicMax(&stats[NTBC_MAX_LEVELS + l], mx);
  }
}

// (s, z) of every level in float32 over the level's range widened to contain 0 (the zero point makes
// real 0 an exact code, Sec. 2.3): lo = min(min, 0), hi = max(max, 0), s = (hi-lo)/255,
// z = clamp(rne(-lo/s), 0, 255); an all-zero level: s = 1, z = 0.
__global__ void k_qat_params(int* __restrict__ stats, int n_levels) {
  const int l = threadIdx.x;
  if (l >= n_levels) return;
  const float lo = fminf(unordered(stats[l]), 0.0f), hi = fmaxf(unordered(stats[NTBC_MAX_LEVELS + l]), 0.0f);
  float s = 1.0f, z = 0.0f;
  if (hi != lo) {
    s = __fdiv_rn(__fsub_rn(hi, lo), 255.0f);
    z = fminf(fmaxf(rintf(__fdiv_rn(-lo, s)), 0.0f), 255.0f);
  }
  reinterpret_cast<float*>(stats)[2 * NTBC_MAX_LEVELS + l] = s;
  stats[3 * NTBC_MAX_LEVELS + l] = (int)z;
}

// Block ids come from the caller; out-of-range ids are clamped into [0, n_positions) so that no input
// can address outside the grid or the targets.
__device__ __forceinline__ int clamp_id(int id, int64_t n_positions) {
  return id < 0 ? 0 : (id >= n_positions ? (int)(n_positions - 1) : id);
}

// Eq. quantizer Q(w) = s (clamp(rne(w/s) + z, 0, 255) - z) and its pass-through mask.
__device__ __forceinline__ float fake_quant(float w, float s, int z, bool* inside) {
  const float t = rintf(__fdiv_rn(w, s)) + (float)z;
  *inside = t >= 0.0f && t <= 255.0f;
  const float q = fminf(fmaxf(t, 0.0f), 255.0f);
  return s * (q - (float)z);
}

struct FeatArgs {
  const float* grid;
  const int* stats;  // null when QAT is off
  const int32_t* ids;
  int64_t n;
  int n_levels, base_res, F, blocks_w, blocks_h;
  int shift_x, shift_y;  // pow2_shift of the block grid, -1: the division path
  int64_t level_offset[NTBC_MAX_LEVELS + 1];
  float* x;          // [n][L*F]
};

// Grid corners and bilinear weights of position p at level l (Eq. grid lookup, cell-centred).
struct Tap {
  int64_t vtx[4];
  float w[4];
};

__device__ __forceinline__ Tap grid_tap_id(const FeatArgs& a, int id, int l) {
  const int bx = id % a.blocks_w, by = id / a.blocks_w;
  const int res = a.base_res << l;
  const dev::Corner cx = a.shift_x >= 0 ? dev::corner_pow2(bx, a.blocks_w, res, a.shift_x) : dev::corner(bx, a.blocks_w, res);
  const dev::Corner cy = a.shift_y >= 0 ? dev::corner_pow2(by, a.blocks_h, res, a.shift_y) : dev::corner(by, a.blocks_h, res);
  const int64_t v00 = a.level_offset[l] + (int64_t)cy.i0 * res + cx.i0;
  Tap t;
  t.vtx[0] = v00;
  t.vtx[1] = v00 + 1;
  t.vtx[2] = v00 + res;
  t.vtx[3] = v00 + res + 1;
  t.w[0] = (1.0f - cx.f) * (1.0f - cy.f);
  t.w[1] = cx.f * (1.0f - cy.f);
  t.w[2] = (1.0f - cx.f) * cy.f;
  t.w[3] = cx.f * cy.f;
  return t;
}

__device__ __forceinline__ Tap grid_tap(const FeatArgs& a, int64_t p, int l) {
  return grid_tap_id(a, clamp_id(a.ids[p], (int64_t)a.blocks_w * a.blocks_h), l);
}

// One thread per (position, level, feature); the F lanes of a (position, level) read the F
// consecutive features of each corner together.
__global__ void __launch_bounds__(kBlock) k_features(FeatArgs a) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= a.n * a.n_levels * a.F) return;
  const int f = (int)(gid % a.F);
  const int64_t pl = gid / a.F;
  const int64_t p = pl / a.n_levels;
  const int l = (int)(pl % a.n_levels);
  const Tap t = grid_tap(a, p, l);
  const float s = a.stats ? reinterpret_cast<const float*>(a.stats)[2 * NTBC_MAX_LEVELS + l] : 1.0f;
  const int z = a.stats ? a.stats[3 * NTBC_MAX_LEVELS + l] : 0;
  float v[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float g = a.grid[t.vtx[c] * a.F + f];
    bool inside;
    v[c] = a.stats ? fake_quant(g, s, z, &inside) : g;
  }
  a.x[pl * a.F + f] = fmaf(t.w[0], v[0], fmaf(t.w[1], v[1], fmaf(t.w[2], v[2], t.w[3] * v[3])));
}

// d_grid[corner] += w_corner * dX (times the pass-through mask of the corner value with QAT), for one
// (position, level, feature).  Acc = float: FP32 atomics (the sum depends on their order).  Acc =
// unsigned long long (deterministic mode): each term is rounded to a fixed-point integer at the step's
// scale (a power of two, *scale) and added with 64-bit integer atomics, whose sum does not depend on
// the order.
template <typename Acc>
__device__ __forceinline__ void scatter_tap(const FeatArgs& a, float df, int id, int l, int f, Acc* __restrict__ dst,
                                            float scale) {
  if (df == 0.0f) return;
  const Tap t = grid_tap_id(a, id, l);
  const float s = a.stats ? reinterpret_cast<const float*>(a.stats)[2 * NTBC_MAX_LEVELS + l] : 1.0f;
  const int z = a.stats ? a.stats[3 * NTBC_MAX_LEVELS + l] : 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (t.w[c] == 0.0f) continue;
    if (a.stats) {
      bool inside;
      fake_quant(a.grid[t.vtx[c] * a.F + f], s, z, &inside);
      if (!inside) continue;
    }
    const float v = t.w[c] * df;
    if constexpr (sizeof(Acc) == 8)
      atomicAdd(&dst[t.vtx[c] * a.F + f], (Acc)(long long)rint((double)v * (double)scale));
    else
      atomicAdd(&dst[t.vtx[c] * a.F + f], v);
  }
}

template <typename Acc>
__device__ __forceinline__ void scatter_one(const FeatArgs& a, const float* __restrict__ dx, int64_t p, int l, int f,
                                            Acc* __restrict__ dst, float scale) {
  const float df = dx[(p * a.n_levels + l) * a.F + f];
  if (df == 0.0f) return;
  scatter_tap<Acc>(a, df, clamp_id(a.ids[p], (int64_t)a.blocks_w * a.blocks_h), l, f, dst, scale);
}

// Levels [first_level, n_levels): one thread per (position, level, feature), feature fastest so that
// the atomics of a corner land in one cache line.
template <typename Acc>
__global__ void __launch_bounds__(kBlock) k_scatter(FeatArgs a, const float* __restrict__ dx, Acc* __restrict__ dgrid,
                                                    int first_level, const float* __restrict__ det_scale) {
  const int nl = a.n_levels - first_level;
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= a.n * nl * a.F) return;
  const int f = (int)(gid % a.F);
  const int64_t pl = gid / a.F;
  scatter_one<Acc>(a, dx, pl / nl, first_level + (int)(pl % nl), f, dgrid, det_scale ? *det_scale : 1.0f);
}

// Levels [first_level, n_levels) when the positions are the texels of whole blocks (16 consecutive
// positions: texels (4bx + x, 4by + y), i = 4y + x, of a texel grid of blocks_w x blocks_h cells) and
// no level is finer than the texel grid: one thread per (block, level, feature).  Adjacent texels'
// corners then differ by at most one vertex, so a block's 16 texels touch at most 5 x 5 vertices of a
// level; their 64 weighted terms are summed in registers first (the bilinear weights are separable:
// sum over y of wy(y, b) * sum over x of wx(x, a) d(x, y)), and the block adds each touched vertex once.
template <typename Acc>
__global__ void __launch_bounds__(kBlock) k_scatter_texels(FeatArgs a, const float* __restrict__ dx,
                                                           Acc* __restrict__ dgrid, int first_level,
                                                           const float* __restrict__ det_scale) {
  const int nl = a.n_levels - first_level;
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= (a.n / 16) * nl * a.F) return;
  const int f = (int)(gid % a.F);
  const int64_t pl = gid / a.F;
  const int l = first_level + (int)(pl % nl);
  const int64_t b = pl / nl;
  const int t0 = clamp_id(a.ids[16 * b], (int64_t)a.blocks_w * a.blocks_h);
  const int tx0 = t0 % a.blocks_w, ty0 = t0 / a.blocks_w;
  const int res = a.base_res << l;
  dev::Corner cx[4], cy[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    cx[k] = a.shift_x >= 0 ? dev::corner_pow2(tx0 + k, a.blocks_w, res, a.shift_x) : dev::corner(tx0 + k, a.blocks_w, res);
    cy[k] = a.shift_y >= 0 ? dev::corner_pow2(ty0 + k, a.blocks_h, res, a.shift_y) : dev::corner(ty0 + k, a.blocks_h, res);
  }
  // rows: T[y][c] = sum over x of wx(x, c) d(x, y), column c = vertex cx[0].i0 + c
  float tr[4][5];
#pragma unroll
  for (int y = 0; y < 4; ++y) {
#pragma unroll
    for (int c = 0; c < 5; ++c) tr[y][c] = 0.0f;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const float d = dx[((16 * b + 4 * y + x) * a.n_levels + l) * a.F + f];
      const int o = cx[x].i0 - cx[0].i0;
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const float w = c == o ? 1.0f - cx[x].f : (c == o + 1 ? cx[x].f : 0.0f);
        tr[y][c] = fmaf(w, d, tr[y][c]);
      }
    }
  }
  const float s = a.stats ? reinterpret_cast<const float*>(a.stats)[2 * NTBC_MAX_LEVELS + l] : 1.0f;
  const int z = a.stats ? a.stats[3 * NTBC_MAX_LEVELS + l] : 0;
  const float scale = det_scale ? *det_scale : 1.0f;
#pragma unroll
  for (int r = 0; r < 5; ++r) {
    float acc[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int o = cy[y].i0 - cy[0].i0;
      const float w = r == o ? 1.0f - cy[y].f : (r == o + 1 ? cy[y].f : 0.0f);
#pragma unroll
      for (int c = 0; c < 5; ++c) acc[c] = fmaf(w, tr[y][c], acc[c]);
    }
    const int vy = cy[0].i0 + r;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const int vx = cx[0].i0 + c;
      if (acc[c] == 0.0f || vx > res - 1 || vy > res - 1) continue;
      const int64_t v = a.level_offset[l] + (int64_t)vy * res + vx;
      if (a.stats) {
        bool inside;
        fake_quant(a.grid[v * a.F + f], s, z, &inside);
        if (!inside) continue;
      }
      if constexpr (sizeof(Acc) == 8)
        atomicAdd(&dgrid[v * a.F + f], (Acc)(long long)rint((double)acc[c] * (double)scale));
      else
        atomicAdd(&dgrid[v * a.F + f], acc[c]);
    }
  }
}

// Levels [0, n_coarse) (their gradient fits in LDS): every block accumulates a contiguous share of the
// batch in LDS and writes its sums to its own row of `part` ([gridDim.x][nv]); k_scatter_reduce then
// adds the rows in block order.  No global atomics, and the sum does not depend on the schedule.
constexpr int kCoarseBlocks = 512;
constexpr int kCoarseThreads = 1024;  // sixteen waves share a block's LDS sums: two blocks fill a CU
constexpr int kCoarseLds = 48 * 1024;

template <typename Acc>
__global__ void __launch_bounds__(kCoarseThreads) k_scatter_coarse(FeatArgs a, const float* __restrict__ dx, Acc* __restrict__ part,
                                                           int n_coarse, const float* __restrict__ det_scale) {
  extern __shared__ __align__(8) unsigned char acc_raw[];
  Acc* acc = reinterpret_cast<Acc*>(acc_raw);
  const float scale = det_scale ? *det_scale : 1.0f;
  const int64_t nv = a.level_offset[n_coarse] * a.F;
  for (int64_t i = threadIdx.x; i < nv; i += kCoarseThreads) acc[i] = (Acc)0;
  __syncthreads();
  const int64_t per_pos = (int64_t)n_coarse * a.F;
  const int64_t total = a.n * per_pos;
  const int64_t share = (total + gridDim.x - 1) / gridDim.x;
  const int64_t e0 = (int64_t)blockIdx.x * share, e1 = e0 + share < total ? e0 + share : total;
  // four elements a round, their loads issued together (the loop is latency-bound otherwise)
  constexpr int kU = 4;
  const int64_t npos = (int64_t)a.blocks_w * a.blocks_h;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += kU * kCoarseThreads) {
    float df[kU];
    int id[kU], lf[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t ee = e + (int64_t)u * kCoarseThreads;
      const bool ok = ee < e1;
      const int64_t p = ok ? ee / per_pos : 0;
      lf[u] = (int)(ee - p * per_pos);
      df[u] = ok ? dx[p * a.n_levels * a.F + lf[u]] : 0.0f;
      id[u] = ok ? a.ids[p] : 0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      scatter_tap<Acc>(a, df[u], clamp_id(id[u], npos), lf[u] / a.F, lf[u] % a.F, acc, scale);
  }
  __syncthreads();
  Acc* row = part + (int64_t)blockIdx.x * nv;
  for (int64_t i = threadIdx.x; i < nv; i += kCoarseThreads) row[i] = acc[i];
}

// dst[i] += sum over the rows of part[rows][nv] in row order: 64 values per block, four row ranges
// per value summed by four thread groups and combined in order.
template <typename Acc>
__global__ void __launch_bounds__(256) k_scatter_reduce(const Acc* __restrict__ part, int rows, int64_t nv,
                                                        Acc* __restrict__ dst) {
  __shared__ Acc sums[4][64];
  const int col = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + col;
  Acc s = (Acc)0;
  if (i < nv) {
    const int r0 = grp * rows / 4, r1 = (grp + 1) * rows / 4;
#pragma unroll 8
    for (int r = r0; r < r1; ++r) s += part[(int64_t)r * nv + i];
  }
  sums[grp][col] = s;
  __syncthreads();
  if (grp == 0 && i < nv) {
    const Acc t = ((sums[0][col] + sums[1][col]) + sums[2][col]) + sums[3][col];
    if (t != (Acc)0) dst[i] += t;
  }
}

// Deterministic mode: the fixed-point scale of a step.  amax = max |dX| over the batch (float bits);
// each grid value sums at most n terms of magnitude <= amax (a position reaches a vertex at most once,
// with a bilinear weight <= 1), so scale = 2^(61 - ceil(log2(n amax))) keeps every partial sum below 2^61.
__global__ void k_absmax_bits(const float* __restrict__ x, int64_t count, unsigned* __restrict__ amax) {
  float m = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(x[i]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) atomicMax(amax, __float_as_uint(m));
}

__global__ void k_det_scale(const unsigned* __restrict__ amax, int64_t n, float* __restrict__ scale) {
  const double m = (double)__uint_as_float(*amax) * (double)n;
  int e = 0;
  if (m > 0.0 && isfinite(m)) {
    frexp(m, &e);  // m < 2^e
    e = 61 - e;
    e = e > 126 ? 126 : (e < -126 ? -126 : e);
  }
  *scale = ldexpf(1.0f, e);
}

// d_grid += fixed-point sums / scale.
__global__ void k_det_finish(unsigned long long* __restrict__ acc, const float* __restrict__ scale, float* __restrict__ d_grid,
                             int64_t count) {
  const double inv = 1.0 / (double)*scale;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const long long v = (long long)acc[i];
    if (v != 0) d_grid[i] += (float)((double)v * inv);
  }
}

__global__ void k_zero_u64(unsigned long long* __restrict__ p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// ------------------------------------------------------------------------------------------ GEMM
enum Epi { EPI_STORE = 0, EPI_BIAS_RELU = 1, EPI_BIAS_SIGMOID = 2, EPI_MASK = 3, EPI_ATOMIC = 4, EPI_BIAS_SELU = 5,
           EPI_SELU_MASK = 6 };

// SELU (the paper's own layout, Sec. 3.4) with the constants of Klambauer et al. (2017).  Its
// derivative from the layer output h = selu(z): lambda where h > 0 (z > 0), otherwise
// lambda alpha e^z = h + lambda alpha; NaN stays NaN in both.
constexpr float kSeluLambda = 1.0507009873554805f;
constexpr float kSeluLambdaAlpha = 1.0507009873554805f * 1.6732632423543772f;
__device__ __forceinline__ float selu_f(float z) { return z > 0.0f ? kSeluLambda * z : kSeluLambdaAlpha * expm1f(z); }
__device__ __forceinline__ float selu_grad_of_out(float h) { return h > 0.0f ? kSeluLambda : h + kSeluLambdaAlpha; }

struct GemmArgs {
  const float* a;
  int64_t sam, sak;  // A(m, k) = a[m*sam + k*sak]
  const float* b;
  int64_t sbk, sbn;  // B(k, n) = b[k*sbk + n*sbn]
  float* c;
  int64_t ldc;
  int M, N, K, k_split;
  const float* bias;  // [N]
  const float* mask;  // C(m, n) *= (mask[m*ldm + n] > 0)
  int64_t ldm;
  float* colsum;      // optional: colsum[m] += sum over k of A(m, k) in FP32 (the bias gradient of a weight product)
};

typedef float f32x4_t __attribute__((ext_vector_type(4)));

// C = A * B with a fused epilogue on the FP32 matrix cores: 64x64 workgroup tile, 16-deep K slices
// staged in LDS; wave w computes the 32x32 quadrant (w/2, w%2) as 2x2 v_mfma_f32_16x16x4f32 tiles
// (operand lane l: row/column l%16, k = l/16; accumulator v of lane l: row 4(l/16)+v, column l%16).
// With g.colsum, the blocks of the first column tile also sum their A rows over their K range from the
// staged slices (one atomic add per row and K range).
template <int EPI>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
  constexpr int TM = 64, TN = 64, TK = 16;
  __shared__ __align__(16) float As[TK][TM + 4];
  __shared__ __align__(16) float Bs[TK][TN + 4];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int kbeg = blockIdx.z * g.k_split;
  const int kend = min(g.K, kbeg + g.k_split);
  f32x4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{};
  const int li = lane & 15, lk = lane >> 4;
  const bool do_cs = g.colsum != nullptr && blockIdx.x == 0 && tid < TM;
  float csum = 0.0f;
  for (int k0 = kbeg; k0 < kend; k0 += TK) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;
      int mm, kk;
      if (g.sak == 1) {
        kk = e % TK;
        mm = e / TK;
      } else {
        mm = e % TM;
        kk = e / TM;
      }
      const int m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < g.M && k < kend) ? g.a[(int64_t)m * g.sam + (int64_t)k * g.sak] : 0.0f;
      int nn, kb;
      if (g.sbn == 1) {
        nn = e % TN;
        kb = e / TN;
      } else {
        kb = e % TK;
        nn = e / TK;
      }
      const int n = n0 + nn, kq = k0 + kb;
      Bs[kb][nn] = (n < g.N && kq < kend) ? g.b[(int64_t)kq * g.sbk + (int64_t)n * g.sbn] : 0.0f;
    }
    __syncthreads();
    if (do_cs) {
#pragma unroll
      for (int kk = 0; kk < TK; ++kk) csum += As[kk][tid];
    }
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const float a0 = As[kk + lk][wm * 32 + li], a1 = As[kk + lk][wm * 32 + 16 + li];
      const float b0 = Bs[kk + lk][wn * 32 + li], b1 = Bs[kk + lk][wn * 32 + 16 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  if (do_cs && m0 + tid < g.M) atomicAdd(&g.colsum[m0 + tid], csum);
#pragma unroll
  for (int tm = 0; tm < 2; ++tm) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + wm * 32 + tm * 16 + 4 * lk + v;
      if (m >= g.M) continue;
#pragma unroll
      for (int tn = 0; tn < 2; ++tn) {
        const int n = n0 + wn * 32 + tn * 16 + li;
        if (n >= g.N) continue;
        const float val = acc[tm][tn][v];
        float* out = g.c + (int64_t)m * g.ldc + n;
        if (EPI == EPI_BIAS_RELU) {
          const float z = val + g.bias[n];
          *out = z < 0.0f ? 0.0f : z;  // ReLU that keeps NaN (so a non-finite parameter is detected)
        } else if (EPI == EPI_BIAS_SIGMOID) {
          *out = 1.0f / (1.0f + expf(-(val + g.bias[n])));
        } else if (EPI == EPI_BIAS_SELU) {
          *out = selu_f(val + g.bias[n]);
        } else if (EPI == EPI_SELU_MASK) {
          *out = val * selu_grad_of_out(g.mask[(int64_t)m * g.ldm + n]);
        } else if (EPI == EPI_MASK) {
          *out = g.mask[(int64_t)m * g.ldm + n] > 0.0f ? val : 0.0f;
        } else if (EPI == EPI_ATOMIC) {
          atomicAdd(out, val);
        } else {
          *out = val;
        }
      }
    }
  }
}

// The same product with bfloat16 operands on the matrix cores (v_mfma_f32_32x32x16_bf16, float32
// accumulation): FP32 operands are rounded to bfloat16 (nearest even) as they are staged in LDS.  A
// block computes a 128 x 128 tile (wave w: the 64 x 64 quadrant (w/2, w%2) as 2 x 2 products of
// 32 x 32); K advances in slices of 32, the next slice's operands loaded into registers while the
// current one is multiplied from LDS (two LDS buffers, one barrier per slice).  LDS holds both
// operands K-contiguous (As[m][k], Bs[n][k]) so each lane's fragment (row or column l%32, K elements
// 8(l/32) .. +7) is one 16-byte read; a K-contiguous source is copied as 8-element runs, an M- or
// N-contiguous source as 4 x 2 blocks transposed into 32-bit pairs.  Accumulator v of lane l is row
// 8(v/4) + 4(l/32) + v%4, column l%32 of its 32 x 32 product.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t bf2(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{lo, hi}, bf16x2_t));
}

constexpr int kBT = 128;         // block tile (rows and columns)
constexpr int kBTK = 32;         // K per slice
constexpr int kBRow = kBTK + 8;  // LDS row stride in bfloat16 (80 bytes)

// One thread's share of a kBT x kBTK operand slice X(r, k) = x[r*sr + k*sk] (r < R, k < kend): two
// groups of eight values, in registers, then written to LDS rows dst[r][k] as bfloat16.
struct Stage {
  float v[2][8];
};

__device__ __forceinline__ void stage_load(Stage& st, const float* __restrict__ x, int64_t sr, int64_t sk, int r0,
                                           int R, int k0, int kend, int tid) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int gi = tid + 256 * q;
    if (sk == 1) {
      // 8 consecutive k: kBT rows x 4 runs
      const int r = gi >> 2, kk = (gi & 3) * 8;
      const int row = r0 + r, k = k0 + kk;
      const float* src = x + (int64_t)row * sr + k;
      if (row < R && k + 8 <= kend && (sr & 3) == 0 && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
        const float4 a = *reinterpret_cast<const float4*>(src), b = *reinterpret_cast<const float4*>(src + 4);
        st.v[q][0] = a.x; st.v[q][1] = a.y; st.v[q][2] = a.z; st.v[q][3] = a.w;
        st.v[q][4] = b.x; st.v[q][5] = b.y; st.v[q][6] = b.z; st.v[q][7] = b.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) st.v[q][e] = (row < R && k + e < kend) ? src[e] : 0.0f;
      }
    } else {
      // 4 consecutive rows x 2 consecutive k: 32 row groups x 16 k pairs
      const int r = (gi & 31) * 4, kk = (gi >> 5) * 2;
      const int row = r0 + r, k = k0 + kk;
      const float* s0 = x + (int64_t)k * sk + row;
      if (sr == 1 && row + 4 <= R && k + 2 <= kend && (sk & 3) == 0 && (reinterpret_cast<uintptr_t>(s0) & 15) == 0) {
        const float4 a = *reinterpret_cast<const float4*>(s0), b = *reinterpret_cast<const float4*>(s0 + sk);
        st.v[q][0] = a.x; st.v[q][1] = a.y; st.v[q][2] = a.z; st.v[q][3] = a.w;
        st.v[q][4] = b.x; st.v[q][5] = b.y; st.v[q][6] = b.z; st.v[q][7] = b.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          st.v[q][e] = (row + e < R && k < kend) ? x[(int64_t)(row + e) * sr + (int64_t)k * sk] : 0.0f;
          st.v[q][4 + e] = (row + e < R && k + 1 < kend) ? x[(int64_t)(row + e) * sr + (int64_t)(k + 1) * sk] : 0.0f;
        }
      }
    }
  }
}

__device__ __forceinline__ void stage_store(const Stage& st, bool kcontig, uint16_t (*dst)[kBRow], int tid) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int gi = tid + 256 * q;
    if (kcontig) {
      const int r = gi >> 2, kk = (gi & 3) * 8;
      *reinterpret_cast<u32x4*>(&dst[r][kk]) =
          u32x4{bf2(st.v[q][0], st.v[q][1]), bf2(st.v[q][2], st.v[q][3]), bf2(st.v[q][4], st.v[q][5]),
                bf2(st.v[q][6], st.v[q][7])};
    } else {
      const int r = (gi & 31) * 4, kk = (gi >> 5) * 2;
#pragma unroll
      for (int e = 0; e < 4; ++e) *reinterpret_cast<uint32_t*>(&dst[r + e][kk]) = bf2(st.v[q][e], st.v[q][4 + e]);
    }
  }
}

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[2][kBT][kBRow];
  __shared__ __align__(16) uint16_t Bs[2][kBT][kBRow];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int tn = blockIdx.x, tm = blockIdx.y, tz = blockIdx.z;
  const int m0 = tm * kBT, n0 = tn * kBT;
  const int kbeg = tz * g.k_split;
  const int kend = min(g.K, kbeg + g.k_split);
  const bool a_k = g.sak == 1, b_k = g.sbk == 1;
  f32x16_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x16_t{};
  const int li = lane & 31, lg = lane >> 5;
  // fused bias gradient (EPI_ATOMIC with colsum, the first column of tiles, A staged MN-contiguous):
  // the thread's A values are rows (tid % 32) * 4 .. +3 of every slice, summed in FP32 before rounding
  const bool rows = EPI == EPI_ATOMIC && g.colsum != nullptr && tn == 0 && !a_k;
  float rs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  auto row_sums = [&](const Stage& st) {
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) rs[e] += st.v[q][e] + st.v[q][4 + e];
  };
  Stage sa, sb;
  if (kbeg < kend) {
    stage_load(sa, g.a, g.sam, g.sak, m0, g.M, kbeg, kend, tid);   // A(m, k)
    stage_load(sb, g.b, g.sbn, g.sbk, n0, g.N, kbeg, kend, tid);   // B(k, n) as rows n
    if (rows) row_sums(sa);
    stage_store(sa, a_k, As[0], tid);
    stage_store(sb, b_k, Bs[0], tid);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += kBTK) {
    const bool more = k0 + kBTK < kend;
    if (more) {
      stage_load(sa, g.a, g.sam, g.sak, m0, g.M, k0 + kBTK, kend, tid);
      stage_load(sb, g.b, g.sbn, g.sbk, n0, g.N, k0 + kBTK, kend, tid);
      if (rows) row_sums(sa);
    }
#pragma unroll
    for (int ks = 0; ks < kBTK / 16; ++ks) {
      u32x4 af[2], bfr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        af[i] = *reinterpret_cast<const u32x4*>(&As[buf][wm * 64 + 32 * i + li][ks * 16 + 8 * lg]);
        bfr[i] = *reinterpret_cast<const u32x4*>(&Bs[buf][wn * 64 + 32 * i + li][ks * 16 + 8 * lg]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, af[i]),
                                                              __builtin_bit_cast(bf16x8_t, bfr[j]), acc[i][j], 0, 0, 0);
    }
    if (more) {
      stage_store(sa, a_k, As[buf ^ 1], tid);
      stage_store(sb, b_k, Bs[buf ^ 1], tid);
    }
    __syncthreads();
    buf ^= 1;
  }
  if (rows) {
    // eight threads hold partial sums of each group of four rows: combine them in LDS (the staging
    // buffers are free after the last barrier of the loop)
    float* part = reinterpret_cast<float*>(&As[0][0][0]);  // [8][kBT]
    const int r = (tid & 31) * 4, grp = tid >> 5;
#pragma unroll
    for (int e = 0; e < 4; ++e) part[grp * kBT + r + e] = rs[e];
    __syncthreads();
    if (tid < kBT && m0 + tid < g.M) {
      float t = 0.0f;
#pragma unroll
      for (int q = 0; q < 8; ++q) t += part[q * kBT + tid];
      atomicAdd(g.colsum + m0 + tid, t);
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int n = n0 + wn * 64 + 32 * j + li;
    if (n >= g.N) continue;
    // the lane's column: its bias read once, rows addressed from one base with 32-bit row offsets
    const float bn = (EPI == EPI_BIAS_RELU || EPI == EPI_BIAS_SIGMOID || EPI == EPI_BIAS_SELU) ? g.bias[n] : 0.0f;
    const int mb = m0 + wm * 64 + 4 * lg;
    float* __restrict__ cb = g.c + (int64_t)mb * g.ldc + n;
    const float* __restrict__ kb = EPI == EPI_MASK || EPI == EPI_SELU_MASK ? g.mask + (int64_t)mb * g.ldm + n : nullptr;
    const int ldc = (int)g.ldc, ldm = (int)g.ldm;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int dm = 32 * i + 8 * (v / 4) + (v % 4);
        if (mb + dm >= g.M) continue;
        const float val = acc[i][j][v];
        float* out = cb + dm * ldc;
        if (EPI == EPI_BIAS_RELU) {
          const float z = val + bn;
          *out = z < 0.0f ? 0.0f : z;  // ReLU that keeps NaN (so a non-finite parameter is detected)
        } else if (EPI == EPI_BIAS_SIGMOID) {
          *out = 1.0f / (1.0f + expf(-(val + bn)));
        } else if (EPI == EPI_BIAS_SELU) {
          *out = selu_f(val + bn);
        } else if (EPI == EPI_SELU_MASK) {
          *out = val * selu_grad_of_out(kb[dm * ldm]);
        } else if (EPI == EPI_MASK) {
          *out = kb[dm * ldm] > 0.0f ? val : 0.0f;
        } else if (EPI == EPI_ATOMIC) {
          atomicAdd(out, val);
        } else {
          *out = val;
        }
      }
    }
  }
}

// Launches the product on the FP32 (bf16 = false) or bfloat16 matrix cores; `splits` K ranges of
// g.k_split each (a multiple of 16 for FP32, of kBTK for bfloat16 unless there is one range).
template <int EPI>
int gemm(const GemmArgs& g, int splits, hipStream_t s, bool bf16 = false) {
  if (bf16) {
    const dim3 grid((unsigned)ceil_div(g.N, kBT), (unsigned)ceil_div(g.M, kBT), (unsigned)splits);
    hipLaunchKernelGGL(k_gemm_bf16<EPI>, grid, dim3(256), 0, s, g);
  } else {
    const dim3 grid((unsigned)ceil_div(g.N, 64), (unsigned)ceil_div(g.M, 64), (unsigned)splits);
    hipLaunchKernelGGL(k_gemm<EPI>, grid, dim3(256), 0, s, g);
  }
  return check_launch("k_gemm");
}

// db[n] += sum over rows of dz[m][n]: a block covers 64 columns of a slice of rows; its four waves
// take every fourth row (coalesced 64-float row segments), then combine in LDS.
__global__ void __launch_bounds__(kBlock) k_colsum(const float* __restrict__ dz, int64_t rows, int cols, int rows_per_block,
                                             float* __restrict__ db) {
  __shared__ float part[4][64];
  const int c = blockIdx.y * 64 + (threadIdx.x & 63);
  const int rg = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(rows, r0 + rows_per_block);
  float acc = 0.0f;
  if (c < cols)
    for (int64_t r = r0 + rg; r < r1; r += 4) acc += dz[r * cols + c];
  part[rg][threadIdx.x & 63] = acc;
  __syncthreads();
  if (rg == 0 && c < cols) atomicAdd(&db[c], part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] + part[3][threadIdx.x]);
}

__global__ void k_dsigmoid(const float* __restrict__ dy, const float* __restrict__ y, float* __restrict__ dz, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dz[i] = dy[i] * y[i] * (1.0f - y[i]);
}

// ------------------------------------------------------------------------------------------ loss
struct LossArgs {
  const float* y;
  float* dy;
  const int32_t* ids;
  int64_t n, n_positions;
  int head_dim, E, C, n_textures, blocks_w;
  int ld;  // floats between the rows of y and dy (head_dim, or the padded width of the fused path)
  int formats[NTBC_MAX_TEXTURES], ep_off[NTBC_MAX_TEXTURES], ch_off[NTBC_MAX_TEXTURES];
  const uint64_t* ref;
  const uint8_t* tex[NTBC_MAX_TEXTURES];
  const uint8_t* btex[NTBC_MAX_TEXTURES];  // block-major copies (texel_row), used when `blocked`
  int blocked;
  float inv_t, t2, w_e, w_c, w_cde, w_cdc;  // t2 = log2(e) / T
  float inv_ne, inv_nc;  // 1/(n E), 1/(n 16 C)
  float* losses;         // [5]
  int dsigmoid;          // write dL/dZ = dL/dY * Y (1 - Y) (the head's pre-activation) instead of dL/dY
  int tex_of[2][NTBC_MAX_TEXTURES];  // the BC1 textures, then the BC4 textures, in head order
  int n_bc1;                         // how many BC1 textures (k_loss_grad_mixed)
};

// Texel row `sub` (4 texels x CH bytes) of block id of texture t: from the block-major copy (the block's
// texels are one contiguous run) when the targets have one, else from the row-major texture.
template <int CH, typename Args>
__device__ __forceinline__ const uint8_t* texel_row(const Args& a, int t, int id, int sub) {
  if (a.blocked) return a.btex[t] + ((int64_t)id * 16 + 4 * sub) * CH;
  const int bx = id % a.blocks_w, by = id / a.blocks_w;
  const int64_t pitch = (int64_t)4 * a.blocks_w * CH;
  return a.tex[t] + (int64_t)(4 * by + sub) * pitch + (int64_t)(4 * bx) * CH;
}

// The gradient written for a head value y: dL/dY, or dL/dZ through the sigmoid.
__device__ __forceinline__ float head_grad(const LossArgs& a, float g, float y) {
  return a.dsigmoid ? g * y * (1.0f - y) : g;
}

// Palette coefficients of logical index n (Eq. palette, Eq. weightBC4): c_n = a e0 + b e1 + k, with
// the weights w_n = n/3 (BC1), n/7 (BC4, e0 > e1) or (n-1)/5 plus the constants 0 and 1 (BC4, e0 <= e1).
// n is a compile-time constant after unrolling, so the mode choice becomes two selects.
template <bool BC1>
__device__ __forceinline__ void palette_coef(bool eight, int n, float* a, float* b, float* k) {
  if (BC1) {
    *b = (float)n * (1.0f / 3.0f);
    *a = 1.0f - *b;
    *k = 0.0f;
    return;
  }
  const float b8 = (float)n * (1.0f / 7.0f);
  const float b6 = (n == 0 || n == 7) ? 0.0f : (float)(n - 1) * 0.2f;
  const float a6 = (n == 0 || n == 7) ? 0.0f : 1.0f - b6;
  *b = eight ? b8 : b6;
  *a = eight ? 1.0f - b8 : a6;
  *k = (!eight && n == 7) ? 1.0f : 0.0f;
}

__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Straight-through decoded-colour term for one texel: distances dist[0..N) (d_n = -dist_n), the
// reference palette pr (built from er0, er1 and the mode) and the texel colour c.  Adds (x - c)^2 to
// *loss for the hard choice x and returns dL/d(d_n) = (1/T) s_n sum_c g_c (pr_n,c - xs_c) with
// g = 2 (x - c) / N_cd, xs = sum_n s_n pr_n, computed as dd_n = (e_n / (T tot)) (G_n - sum_m e_m G_m / tot)
// with e_n = exp(-(dist_n - dist_min) / T), tot = sum e_n and G_n = g . pr_n.  t2 = log2(e) / T.
template <int CH, int N>
__device__ __forceinline__ void cd_term(const float* dist, const float (*pr)[3], const float* er0, const float* er1,
                                        bool eight_ref, const float* c, float inv_ncd, float inv_t, float t2,
                                        float* loss, float* dd) {
#pragma clang fp contract(fast)
  // hard choice: the first nearest entry k.  Its colour is rebuilt from k with the same operations
  // that built pr (an indexed read of pr would force the palette out of registers).
  int k = 0;
  float dmin = dist[0];
#pragma unroll
  for (int n = 1; n < N; ++n) {
    const bool nearer = dist[n] < dmin;
    dmin = nearer ? dist[n] : dmin;
    k = nearer ? n : k;
  }
  float ak, bk, kk;
  palette_coef<CH == 3>(eight_ref, k, &ak, &bk, &kk);
  float gx[CH];
#pragma unroll
  for (int ch = 0; ch < CH; ++ch) {
    const float d = (ak * er0[ch] + bk * er1[ch] + kk) - c[ch];
    *loss += d * d;
    gx[ch] = 2.0f * d * inv_ncd;
  }
  float e[N], G[N], tot = 0.0f, gsum = 0.0f;
#pragma unroll
  for (int n = 0; n < N; ++n) {
    e[n] = __builtin_amdgcn_exp2f((dmin - dist[n]) * t2);
    tot += e[n];
    float g = gx[0] * pr[n][0];
#pragma unroll
    for (int ch = 1; ch < CH; ++ch) g += gx[ch] * pr[n][ch];
    G[n] = g;
    gsum += e[n] * g;
  }
  const float r = fast_rcp(tot);
  const float gbar = gsum * r, scale = inv_t * r;
#pragma unroll
  for (int n = 0; n < N; ++n) dd[n] = e[n] * scale * (G[n] - gbar);
}

// Losses and head gradients of one texture of one position, for the texel row `sub` (texels
// 4*sub .. 4*sub+3; four lanes share a position/texture).  Returns the partial endpoint gradients in
// de0/de1; lane sub == 0 also carries the L_e term.  The caller combines the four lanes and writes the
// endpoint gradients.  Non-finite heads show up as non-finite gradients, which the caller checks.  A
// distance ||v|| and its unit vector come from one reciprocal square root (CH = 3), or from |v| and
// sign(v) (CH = 1: no transcendental).
template <int CH>
__device__ __forceinline__ void texture_loss(const LossArgs& a, int64_t p, int t, int id, int sub, float* le, float* lc,
                                             float* lcde, float* lcdc, bool* bad, float de0[3], float de1[3]) {
#pragma clang fp contract(fast)
  constexpr bool bc1 = CH == 3;
  constexpr int N = bc1 ? 4 : 8;
  const float* yp = a.y + p * a.ld;
  float* dyp = a.dy + p * a.ld;
  const uint64_t w = a.ref[(int64_t)t * a.n_positions + id];
  float er0[3] = {0, 0, 0}, er1[3] = {0, 0, 0};
  bool eight_ref = true;
  constexpr float k255 = 1.0f / 255.0f;
  if (bc1) {
    const uint32_t c0 = (uint32_t)(w & 0xFFFF), c1 = (uint32_t)((w >> 16) & 0xFFFF);
    er0[0] = (float)dev::expand5d((c0 >> 11) & 31) * k255;
    er0[1] = (float)dev::expand6d((c0 >> 5) & 63) * k255;
    er0[2] = (float)dev::expand5d(c0 & 31) * k255;
    er1[0] = (float)dev::expand5d((c1 >> 11) & 31) * k255;
    er1[1] = (float)dev::expand6d((c1 >> 5) & 63) * k255;
    er1[2] = (float)dev::expand5d(c1 & 31) * k255;
  } else {
    const int b0 = (int)(w & 0xFF), b1 = (int)((w >> 8) & 0xFF);
    er0[0] = (float)b0 * k255;
    er1[0] = (float)b1 * k255;
    eight_ref = b0 > b1;
  }
  float pr[N][3], ph[N][3], ca[N], cb[N];
  const int e = a.ep_off[t];
  float eh0[3], eh1[3];
#pragma unroll
  for (int ch = 0; ch < CH; ++ch) {
    eh0[ch] = yp[e + ch];
    eh1[ch] = yp[e + CH + ch];
  }
  // the predicted colours of the lane's four texels, loaded before the palettes are built
  float chat4[4][CH];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) chat4[x][ch] = yp[a.E + (4 * sub + x) * a.C + a.ch_off[t] + ch];
  const bool eight_hat = bc1 ? true : eh0[0] > eh1[0];
#pragma unroll
  for (int n = 0; n < N; ++n) {
    float ar, br, kr;
    palette_coef<bc1>(eight_ref, n, &ar, &br, &kr);
    float ah, bh, kh;
    palette_coef<bc1>(eight_hat, n, &ah, &bh, &kh);
    ca[n] = ah;
    cb[n] = bh;
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
      pr[n][ch] = ar * er0[ch] + br * er1[ch] + kr;
      ph[n][ch] = ah * eh0[ch] + bh * eh1[ch] + kh;
    }
  }
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) de0[ch] = de1[ch] = 0.0f;
  if (sub == 0) {
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
      const float d0 = eh0[ch] - er0[ch], d1 = eh1[ch] - er1[ch];
      *le += d0 * d0 + d1 * d1;
      de0[ch] = a.w_e * 2.0f * d0 * a.inv_ne;
      de1[ch] = a.w_e * 2.0f * d1 * a.inv_ne;
    }
  }
  const uint8_t* row = texel_row<CH>(a, t, id, sub);
  // the lane's texel row (4 texels x CH bytes) in CH words: dword loads when the texture is 4-byte
  // aligned (the row offset always is), byte loads otherwise
  uint32_t rw[CH];
  if ((reinterpret_cast<uintptr_t>(row) & 3) == 0) {
#pragma unroll
    for (int k = 0; k < CH; ++k) rw[k] = reinterpret_cast<const uint32_t*>(row)[k];
  } else {
#pragma unroll
    for (int k = 0; k < CH; ++k)
      rw[k] = (uint32_t)row[4 * k] | ((uint32_t)row[4 * k + 1] << 8) | ((uint32_t)row[4 * k + 2] << 16) |
              ((uint32_t)row[4 * k + 3] << 24);
  }
#pragma unroll 1
  for (int x = 0; x < 4; ++x) {
    const int i = 4 * sub + x;
    float c[CH], chat[CH], dchat[CH];
    const int ci = a.E + i * a.C + a.ch_off[t];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
      const int b = x * CH + ch;  // byte of the row (run-time x: words chosen by selects, no indexing)
      const uint32_t word = CH == 1 ? rw[0] : (b < 4 ? rw[0] : (b < 8 ? rw[CH > 1 ? 1 : 0] : rw[CH > 2 ? 2 : 0]));
      c[ch] = (float)((word >> (8 * (b & 3))) & 255u) * k255;
      chat[ch] = x == 0 ? chat4[0][ch] : (x == 1 ? chat4[1][ch] : (x == 2 ? chat4[2][ch] : chat4[3][ch]));
      const float d = chat[ch] - c[ch];
      *lc += d * d;
      dchat[ch] = a.w_c * 2.0f * d * a.inv_nc;
    }
    // endpoint branch: d_n = -||c - c^_n|| over the palette of the predicted endpoints
    float dist[N], unit[N], dd[N];  // unit: 1/dist (CH = 3) or sign(c - c^_n) (CH = 1)
#pragma unroll
    for (int n = 0; n < N; ++n) {
      if (CH == 1) {
        const float v = c[0] - ph[n][0];
        dist[n] = fabsf(v);
        unit[n] = v > 0.0f ? 1.0f : (v < 0.0f ? -1.0f : 0.0f);
      } else {
        float acc = 0.0f;
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) {
          const float d = c[ch] - ph[n][ch];
          acc += d * d;
        }
        const float rs = acc > 0.0f ? __builtin_amdgcn_rsqf(acc) : 0.0f;
        dist[n] = acc * rs;
        unit[n] = rs;
      }
    }
    cd_term<CH, N>(dist, pr, er0, er1, eight_ref, c, a.inv_nc, a.inv_t, a.t2, lcde, dd);
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const float q = a.w_cde * dd[n] * unit[n];
      const float qa = q * ca[n], qb = q * cb[n];
      if (CH == 1) {
        de0[0] += qa;
        de1[0] += qb;
      } else {
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) {
          const float v = c[ch] - ph[n][ch];
          de0[ch] += qa * v;
          de1[ch] += qb * v;
        }
      }
    }
    // colour branch: d_n = -||c^ - c_n|| over the reference palette
#pragma unroll
    for (int n = 0; n < N; ++n) {
      if (CH == 1) {
        const float v = chat[0] - pr[n][0];
        dist[n] = fabsf(v);
        unit[n] = v > 0.0f ? 1.0f : (v < 0.0f ? -1.0f : 0.0f);
      } else {
        float acc = 0.0f;
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) {
          const float d = chat[ch] - pr[n][ch];
          acc += d * d;
        }
        const float rs = acc > 0.0f ? __builtin_amdgcn_rsqf(acc) : 0.0f;
        dist[n] = acc * rs;
        unit[n] = rs;
      }
    }
    cd_term<CH, N>(dist, pr, er0, er1, eight_ref, c, a.inv_nc, a.inv_t, a.t2, lcdc, dd);
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const float q = a.w_cdc * dd[n] * unit[n];
      if (CH == 1) {
        dchat[0] -= q;
      } else {
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) dchat[ch] -= q * (chat[ch] - pr[n][ch]);
      }
    }
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
      dyp[ci + ch] = head_grad(a, dchat[ch], chat[ch]);
      *bad |= !isfinite(dchat[ch]);
    }
  }
}

// Four lanes per (texture, position).  A block has one wave per texture (so a wave works on one
// format) and covers 16 positions at a time: the waves of a block read the same rows of the heads and
// write the same rows of their gradient at about the same time, so those rows pass through L2 once
// instead of once per texture.  A grid-stride loop over groups of 16 positions keeps the shuffles
// uniform; the loss sums are reduced per block and added with one atomic per block and loss
// (same-address atomics from every wave serialise in L2).
// Blocks of the loss launches: every block resident at once (a CU holds 16 of their waves at four waves
// per SIMD; a block has one wave per texture), so the grid-stride loop has no second, thinly filled round.
int loss_blocks(int64_t n, int waves_per_block) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      cus = v > 0 ? v : 256;
    else
      cus = 256;
  }
  const int64_t resident = (int64_t)cus * std::max(1, 16 / std::max(1, waves_per_block));
  return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 16), resident));
}

// The wave's groups of 16 positions for texture t of format CH (CH = 3: BC1, CH = 1: BC4); the loss sums
// accumulate in le .. lcdc, non-finite gradients in bad.
template <int CH>
__device__ __forceinline__ void loss_groups(const LossArgs& a, int t, int lane, float& le, float& lc, float& lcde,
                                            float& lcdc, bool& bad) {
  const int64_t groups = (a.n + 15) / 16;
  for (int64_t grp = blockIdx.x; grp < groups; grp += gridDim.x) {
    float de0[3] = {0, 0, 0}, de1[3] = {0, 0, 0};
    const int64_t p = grp * 16 + (lane >> 2);
    const int sub = lane & 3;
    const bool active = p < a.n;
    if (active) {
      const int id = clamp_id(a.ids[p], a.n_positions);
      texture_loss<CH>(a, p, t, id, sub, &le, &lc, &lcde, &lcdc, &bad, de0, de1);
    }
    // combine the endpoint gradients of the four lanes of a position (an aligned group of the wave)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
#pragma unroll
      for (int off = 1; off < 4; off <<= 1) {
        de0[ch] += __shfl_xor(de0[ch], off);
        de1[ch] += __shfl_xor(de1[ch], off);
      }
    }
    if (active && sub == 0) {
      constexpr int ch_n = CH;
      float* dyp = a.dy + p * a.ld + a.ep_off[t];
      const float* yp = a.y + p * a.ld + a.ep_off[t];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        if (ch < ch_n) {
          dyp[ch] = head_grad(a, de0[ch], yp[ch]);
          dyp[ch_n + ch] = head_grad(a, de1[ch], yp[ch_n + ch]);
          bad |= !isfinite(de0[ch]) || !isfinite(de1[ch]);
        }
      }
    }
  }
}

// Block-reduced loss sums: one atomic add per block and loss, the skip flag when any wave saw a
// non-finite value.
__device__ __forceinline__ void loss_finish(const LossArgs& a, float le, float lc, float lcde, float lcdc, bool bad,
                                            float (*part)[4], int* part_bad) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    le += __shfl_xor(le, off);
    lc += __shfl_xor(lc, off);
    lcde += __shfl_xor(lcde, off);
    lcdc += __shfl_xor(lcdc, off);
  }
  const unsigned long long anybad = __ballot(bad);
  if (lane == 0) {
    part[wave][0] = le;
    part[wave][1] = lc;
    part[wave][2] = lcde;
    part[wave][3] = lcdc;
    part_bad[wave] = anybad != 0;
  }
  __syncthreads();
  const int n_waves = (int)(blockDim.x / 64);
  if (threadIdx.x < 4) {
    float s = 0.0f;
    for (int w = 0; w < n_waves; ++w) s += part[w][threadIdx.x];
    const float scale = threadIdx.x == 0 ? a.inv_ne : a.inv_nc;
    atomicAdd(&a.losses[threadIdx.x], s * scale);
  } else if (threadIdx.x == 4) {
    int any = 0;
    for (int w = 0; w < n_waves; ++w) any |= part_bad[w];
    if (any) atomicExch(&a.losses[4], 1.0f);
  }
}

// Materials of one format: the block has one wave per texture (wave w works on texture
// a.tex_of[CH == 3 ? 0 : 1][w]).
template <int CH>
__global__ void __launch_bounds__(64 * NTBC_MAX_TEXTURES) k_loss_grad(LossArgs a) {
  __shared__ float part[NTBC_MAX_TEXTURES][4];
  __shared__ int part_bad[NTBC_MAX_TEXTURES];
  float le = 0.0f, lc = 0.0f, lcde = 0.0f, lcdc = 0.0f;
  bool bad = false;
  loss_groups<CH>(a, a.tex_of[CH == 3 ? 0 : 1][threadIdx.x >> 6], threadIdx.x & 63, le, lc, lcde, lcdc, bad);
  loss_finish(a, le, lc, lcde, lcdc, bad, part, part_bad);
}

// Materials of both formats: waves 0 .. n_bc1-1 take the BC1 textures, the others the BC4 textures (a
// wave-uniform branch), so the waves of a block read each row of the heads together.
__global__ void __launch_bounds__(64 * NTBC_MAX_TEXTURES) k_loss_grad_mixed(LossArgs a) {
  __shared__ float part[NTBC_MAX_TEXTURES][4];
  __shared__ int part_bad[NTBC_MAX_TEXTURES];
  float le = 0.0f, lc = 0.0f, lcde = 0.0f, lcdc = 0.0f;
  bool bad = false;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (wave < a.n_bc1) loss_groups<3>(a, a.tex_of[0][wave], lane, le, lc, lcde, lcdc, bad);
  else loss_groups<1>(a, a.tex_of[1][wave - a.n_bc1], lane, le, lc, lcde, lcdc, bad);
  loss_finish(a, le, lc, lcde, lcdc, bad, part, part_bad);
}

// ------------------------------------------------------------------------------------------ naive loss
// Naive approach (Sec. 3.1): the weight head holds texel i's weight of texture t at E + i*T + t.
struct NaiveLossArgs {
  const float* y;
  float* dy;
  const int32_t* ids;
  int64_t n, n_positions;
  int ld, E, T, blocks_w;
  int formats[NTBC_MAX_TEXTURES], ep_off[NTBC_MAX_TEXTURES];
  const uint8_t* tex[NTBC_MAX_TEXTURES];
  const uint8_t* btex[NTBC_MAX_TEXTURES];  // block-major copies (texel_row), used when `blocked`
  int blocked;
  float inv_n;     // 1 / (n 16 C)
  float* losses;   // [5]
  int dsigmoid;    // write dL/dZ through the sigmoid instead of dL/dY
  int stage;       // 1: continuous weights; 2: the quantised weights w_n, no weight gradient
};

// One texture of one position, texel row `sub`: decoded colours x = (1 - w) e0^ + w e1^, the squared
// error against the texels, the weight gradients (stage 1) and the partial endpoint gradients.
template <int CH>
__device__ __forceinline__ void naive_texture_loss(const NaiveLossArgs& a, int64_t p, int t, int id, int sub, float* loss,
                                                   bool* bad, float de0[3], float de1[3]) {
  const float* yp = a.y + p * a.ld;
  float* dyp = a.dy + p * a.ld;
  const int e = a.ep_off[t];
  float eh0[3] = {0, 0, 0}, eh1[3] = {0, 0, 0};
#pragma unroll
  for (int ch = 0; ch < CH; ++ch) {
    eh0[ch] = yp[e + ch];
    eh1[ch] = yp[e + CH + ch];
  }
  const bool eight = CH == 3 ? true : eh0[0] > eh1[0];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) de0[ch] = de1[ch] = 0.0f;
  const uint8_t* row = texel_row<CH>(a, t, id, sub);
  constexpr float k255 = 1.0f / 255.0f;
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int i = 4 * sub + x;
    const int wi = a.E + i * a.T + t;
    const float w = yp[wi];
    float wq = w;
    if (a.stage == 2) {
      if (CH == 3)
        dev::naive_index_bc1(w, &wq);
      else
        dev::naive_index_bc4(w, eight, &wq);
    }
    float dw = 0.0f;
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
      const float c = (float)row[x * CH + ch] * k255;
      const float r = (1.0f - wq) * eh0[ch] + wq * eh1[ch] - c;
      *loss += r * r;
      const float g = 2.0f * r * a.inv_n;
      de0[ch] += g * (1.0f - wq);
      de1[ch] += g * wq;
      dw += g * (eh1[ch] - eh0[ch]);
    }
    const float gw = a.stage == 1 ? dw : 0.0f;
    dyp[wi] = a.dsigmoid ? gw * w * (1.0f - w) : gw;
    *bad |= !isfinite(dw);
  }
}

// Four lanes per (texture, position), one wave per texture, as k_loss_grad.
__global__ void __launch_bounds__(64 * NTBC_MAX_TEXTURES) k_loss_naive(NaiveLossArgs a) {
  __shared__ float part[NTBC_MAX_TEXTURES];
  __shared__ int part_bad[NTBC_MAX_TEXTURES];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = wave;
  const int64_t groups = (a.n + 15) / 16;
  float loss = 0.0f;
  bool bad = false;
  for (int64_t grp = blockIdx.x; grp < groups; grp += gridDim.x) {
    float de0[3] = {0, 0, 0}, de1[3] = {0, 0, 0};
    const int64_t p = grp * 16 + (lane >> 2);
    const int sub = lane & 3;
    const bool active = p < a.n;
    if (active) {
      const int id = clamp_id(a.ids[p], a.n_positions);
      if (a.formats[t] == NTBC_BC1)
        naive_texture_loss<3>(a, p, t, id, sub, &loss, &bad, de0, de1);
      else
        naive_texture_loss<1>(a, p, t, id, sub, &loss, &bad, de0, de1);
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
#pragma unroll
      for (int off = 1; off < 4; off <<= 1) {
        de0[ch] += __shfl_xor(de0[ch], off);
        de1[ch] += __shfl_xor(de1[ch], off);
      }
    }
    if (active && sub == 0) {
      const int ch_n = a.formats[t] == NTBC_BC1 ? 3 : 1;
      float* dyp = a.dy + p * a.ld + a.ep_off[t];
      const float* yp = a.y + p * a.ld + a.ep_off[t];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        if (ch < ch_n) {
          const float y0 = yp[ch], y1 = yp[ch_n + ch];
          dyp[ch] = a.dsigmoid ? de0[ch] * y0 * (1.0f - y0) : de0[ch];
          dyp[ch_n + ch] = a.dsigmoid ? de1[ch] * y1 * (1.0f - y1) : de1[ch];
          bad |= !isfinite(de0[ch]) || !isfinite(de1[ch]);
        }
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off);
  const unsigned long long anybad = __ballot(bad);
  if (lane == 0) {
    part[wave] = loss;
    part_bad[wave] = anybad != 0;
  }
  __syncthreads();
  const int n_waves = (int)(blockDim.x / 64);
  if (threadIdx.x == 0) {
    float sum = 0.0f;
    int any = 0;
    for (int w = 0; w < n_waves; ++w) {
      sum += part[w];
      any |= part_bad[w];
    }
    atomicAdd(&a.losses[0], sum * a.inv_n);
    if (any) atomicExch(&a.losses[4], 1.0f);
  }
}

// Sets flag[0] = 1 if any of x[0..n) is not finite.
__global__ void k_check_finite(const float* __restrict__ x, int64_t n, float* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicExch(flag, 1.0f);
}

// ------------------------------------------------------------------------------------------ Adam
struct AdamArgs {
  float b1, b2, eps, bc1, bc2;  // bc = 1 / (1 - beta^t); the learning rates come with the ranges

  const float* flag;                // skip when *flag != 0
};

// One parameter range of an Adam launch, with its learning rate; `blocks` of the launch work on it.
struct AdamPart {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t n;
  float lr;
  int blocks;
};

__device__ __forceinline__ void adam1(float& p, float g, float& m, float& v, float lr, const AdamArgs& a) {
  const float mi = a.b1 * m + (1.0f - a.b1) * g;
  const float vi = a.b2 * v + (1.0f - a.b2) * g * g;
  m = mi;
  v = vi;
  p -= lr * (mi * a.bc1) / (sqrtf(vi * a.bc2) + a.eps);
}

// Adam over two parameter ranges in one launch: blocks [0, x.blocks) update x, the others y (an empty
// y has no blocks).  A range whose four arrays are 16-byte aligned moves in 16-byte words with
// non-temporal loads and stores (each word is touched once a step, and streaming the grid's moments
// through the caches would evict what the next step's kernels read), its < 4 trailing elements singly;
// any other range element by element.  The arithmetic per element is the same either way.
__global__ void __launch_bounds__(256) k_adam(AdamPart x, AdamPart y, AdamArgs a) {
  if (*a.flag != 0.0f) return;
  const bool first = blockIdx.x < (unsigned)x.blocks;
  const AdamPart& r = first ? x : y;
  const int64_t b = first ? blockIdx.x : blockIdx.x - x.blocks;
  const int64_t t = b * blockDim.x + threadIdx.x, stride = (int64_t)r.blocks * blockDim.x;
  const bool vec = ((reinterpret_cast<uintptr_t>(r.p) | reinterpret_cast<uintptr_t>(r.g) | reinterpret_cast<uintptr_t>(r.m) |
                     reinterpret_cast<uintptr_t>(r.v)) & 15) == 0;
  int64_t done = 0;
  if (vec) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int64_t n4 = r.n / 4;
    f4* p4 = reinterpret_cast<f4*>(r.p);
    const f4* g4 = reinterpret_cast<const f4*>(r.g);
    f4* m4 = reinterpret_cast<f4*>(r.m);
    f4* v4 = reinterpret_cast<f4*>(r.v);
    for (int64_t i = t; i < n4; i += stride) {
      const f4 p0 = __builtin_nontemporal_load(p4 + i), g0 = __builtin_nontemporal_load(g4 + i);
      const f4 m0 = __builtin_nontemporal_load(m4 + i), v0 = __builtin_nontemporal_load(v4 + i);
      float pp[4] = {p0.x, p0.y, p0.z, p0.w}, mm[4] = {m0.x, m0.y, m0.z, m0.w}, vv[4] = {v0.x, v0.y, v0.z, v0.w};
      const float gg[4] = {g0.x, g0.y, g0.z, g0.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) adam1(pp[e], gg[e], mm[e], vv[e], r.lr, a);
      __builtin_nontemporal_store(f4{pp[0], pp[1], pp[2], pp[3]}, p4 + i);
      __builtin_nontemporal_store(f4{mm[0], mm[1], mm[2], mm[3]}, m4 + i);
      __builtin_nontemporal_store(f4{vv[0], vv[1], vv[2], vv[3]}, v4 + i);
    }
    done = 4 * n4;
  }
  for (int64_t i = done + t; i < r.n; i += stride) adam1(r.p[i], r.g[i], r.m[i], r.v[i], r.lr, a);
}

// Launches k_adam over ranges x and y (y.n = 0: x alone).
int adam(AdamPart x, AdamPart y, const AdamArgs& a, hipStream_t strm) {
  auto blocks_of = [](int64_t n) { return n > 0 ? (int)std::min<int64_t>(ceil_div(ceil_div(n, 4), 256), 8192) : 0; };
  x.blocks = blocks_of(x.n);
  y.blocks = blocks_of(y.n);
  if (x.blocks + y.blocks == 0) return NTBC_OK;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)(x.blocks + y.blocks)), dim3(256), 0, strm, x, y, a);
  return check_launch("k_adam");
}

// ------------------------------------------------------------------------------------------ quantise
__global__ void k_quantize(const float* __restrict__ g, LevelArgs la, const int* __restrict__ stats,
                           uint8_t* __restrict__ codes) {
  const int l = blockIdx.y;
  if (l >= la.n_levels) return;
  const float s = reinterpret_cast<const float*>(stats)[2 * NTBC_MAX_LEVELS + l];
  const int z = stats[3 * NTBC_MAX_LEVELS + l];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < la.count[l]; i += (int64_t)gridDim.x * blockDim.x) {
    const float t = rintf(__fdiv_rn(g[la.begin[l] + i], s)) + (float)z;
    codes[la.begin[l] + i] = (uint8_t)fminf(fmaxf(t, 0.0f), 255.0f);
  }
}

__global__ void k_export_qparams(const int* __restrict__ stats, int n_levels, float* __restrict__ scale, int32_t* __restrict__ zero) {
  const int l = threadIdx.x;
  if (l < n_levels) {
    scale[l] = reinterpret_cast<const float*>(stats)[2 * NTBC_MAX_LEVELS + l];
    zero[l] = stats[3 * NTBC_MAX_LEVELS + l];
  }
}

// ================================================================================== fused bfloat16
// The bfloat16 training step with the layers chained in registers (the inference kernel's layout):
//
//   k_pack_train   FP32 weights -> bfloat16 A operands of the forward products (W_k) and of the
//                  backward products (W_k^T), biases padded to whole tiles
//   k_train_fwd    per 128 positions: (fake-quantised) grid features -> hidden layers -> sigmoid heads,
//                  activations never leave registers between layers; writes the heads, the ReLU
//                  masks (one bit per activation) and the bfloat16 layer inputs position-contiguous
//                  ([neuron][position], the K-major operand of the weight gradient)
//   k_loss_grad    dL/dZ of the head (as for the unfused step)
//   k_train_bwd    per 128 positions: dZ_head -> dZ_k = (W_{k+1}^T dZ_{k+1}) * mask_k down to
//                  dX = W_0^T dZ_0, chained in registers like the forward; writes every dZ_k
//                  position-contiguous in bfloat16 and dX in FP32 for the grid scatter
//   k_train_dw     dW_k = dZ_k^T H_{k-1} and db_k = sum over positions of dZ_k for every layer in
//                  one launch: 128 x 128 output tiles, the batch split into K ranges, FP32 partial
//                  tiles reduced in a fixed order by k_train_dw_reduce (no atomics: deterministic)
//
// Lane (j, g) of a wave owns position j of the wave's 32 and row group g, as in the inference kernel:
// accumulator v of output tile t is neuron 32t + 8(v/4) + 4g + v%4; values 8h..8h+7 of tile t are the
// B operand of K-step 2t+h of the next product.  The backward products use the same layout with
// W_k^T as the A operand, so the masks of the forward apply to the backward accumulators lane by lane.
constexpr int kFW = 4;            // waves per workgroup: 128 positions
constexpr int kFPos = 32 * kFW;
constexpr int kFThreads = 64 * kFW;
constexpr int kFChunkTiles = 2;   // output tiles per weight chunk
constexpr int kFMaxChunks = 48;
constexpr int kFMaxLayers = 5;
constexpr int kFHeadTiles = 6;    // head rows padded to at most 192
constexpr int kFHeadLd = 32 * kFHeadTiles;
constexpr int kFPrefetch = 4;

struct FChunks {
  int n;
  int cap;                   // u32x4 slots of one chunk buffer
  int64_t src[kFMaxChunks];  // u32x4 offset into the packed weights
  int len[kFMaxChunks];
};

__device__ __forceinline__ uint32_t fbf2(float lo, float hi) { return bf2(lo, hi); }

__device__ __forceinline__ u32x4 fpack8(const float* v) {
  return u32x4{fbf2(v[0], v[1]), fbf2(v[2], v[3]), fbf2(v[4], v[5]), fbf2(v[6], v[7])};
}

__device__ __forceinline__ uint16_t fbf1(float x) { return (uint16_t)(fbf2(x, 0.0f) & 0xFFFFu); }

// Sigmoid from the hardware exp2 and reciprocal (each within about one ulp): |error| < 3e-7 for |z| < 64,
// far inside the bfloat16 products' rounding.
__device__ __forceinline__ float fsigmoid(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-z * 1.4426950408889634f));
}

__device__ __forceinline__ f32x16_t fmma(const u32x4& a, const u32x4& b, const f32x16_t& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                 0, 0, 0);
}

__device__ __forceinline__ void fwait_dma() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Copies chunk c of the packed weights into LDS buffer dst (direct global -> LDS, 16 bytes a lane).
__device__ __forceinline__ void fchunk_dma(const u32x4* __restrict__ wp, const FChunks& ct, int c, u32x4* dst, int tid) {
  if (c >= ct.n) return;
  const int wave_base = __builtin_amdgcn_readfirstlane(tid & ~63);
  const int len = ct.len[c];
  const u32x4* src = wp + ct.src[c];
  for (int r = 0; r * kFThreads < len; ++r) {
    const int e = tid + kFThreads * r;
    if (e < len)
      __builtin_amdgcn_global_load_lds(src + e, (__attribute__((address_space(3))) void*)(dst + wave_base + kFThreads * r),
                                       16, 0, 0);
  }
}

// Products of up to two output tiles over KS K-steps from an LDS chunk (A fragment of tile u, step s,
// lane l at wb[(u*KS + s)*64 + l]), the fragments read kFPrefetch steps ahead.
template <int KS, int NB>
__device__ __forceinline__ void fchunk_mfma(const u32x4* wb, const u32x4 (&b)[NB], int lane, int valid,
                                            f32x16_t (&acc)[kFChunkTiles]) {
  static_assert(KS <= NB, "operand count");
  constexpr int PD = kFPrefetch < KS ? kFPrefetch : KS;
  u32x4 ring[PD][kFChunkTiles];
#pragma unroll
  for (int d = 0; d < PD; ++d)
#pragma unroll
    for (int u = 0; u < kFChunkTiles; ++u) ring[d][u] = u < valid ? wb[(u * KS + d) * 64 + lane] : u32x4{};
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    u32x4 cur[kFChunkTiles];
#pragma unroll
    for (int u = 0; u < kFChunkTiles; ++u) cur[u] = ring[s % PD][u];
    if (s + PD < KS) {
#pragma unroll
      for (int u = 0; u < kFChunkTiles; ++u)
        if (u < valid) ring[s % PD][u] = wb[(u * KS + s + PD) * 64 + lane];
    }
#pragma unroll
    for (int u = 0; u < kFChunkTiles; ++u)
      if (u < valid) acc[u] = fmma(cur[u], b[s], acc[u]);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// ----------------------------------------------------------------------------- weight packing
struct PackTrainArgs {
  const float* w;  // canonical FP32 weights
  int n_layers;
  int in_dim[kFMaxLayers], out_dim[kFMaxLayers];
  int64_t w_off[kFMaxLayers], b_off[kFMaxLayers];
  // forward: A(row = output neuron, K = layer input), rows padded to otiles*32, K to ksteps*16
  int f_otiles[kFMaxLayers], f_ksteps[kFMaxLayers];
  int64_t f_off[kFMaxLayers];
  // backward: A(row = layer input neuron, K = output neuron)
  int b_otiles[kFMaxLayers], b_ksteps[kFMaxLayers];
  int64_t b_off2[kFMaxLayers];
  int bias_off[kFMaxLayers];  // padded biases (floats)
  u32x4* pack;
  float* bias;
  float* zero5;  // when set, block (0, 0) zeroes these five floats (a training step's loss sums and flag)
};

// K index of element m of K-step s in lane group g: the grid features (forward layer 0) and the head
// gradient (backward of the head, read from memory) are in natural order; a chained input (the
// previous product's accumulators) is permuted.
__device__ __forceinline__ int fk_natural(int s, int g, int m) { return 16 * s + 8 * g + m; }
__device__ __forceinline__ int fk_chained(int s, int g, int m) {
  return 32 * (s / 2) + 16 * (s % 2) + 8 * (m / 4) + 4 * g + (m % 4);
}

__global__ void __launch_bounds__(256) k_pack_train(PackTrainArgs a) {
  if (a.zero5 != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 5) a.zero5[threadIdx.x] = 0.0f;
  const int layer = blockIdx.y >> 1;
  const bool bwd = (blockIdx.y & 1) != 0;
  if (layer >= a.n_layers) return;
  const int in = a.in_dim[layer], out = a.out_dim[layer];
  const float* w = a.w + a.w_off[layer];
  const int ot = bwd ? a.b_otiles[layer] : a.f_otiles[layer];
  const int ks = bwd ? a.b_ksteps[layer] : a.f_ksteps[layer];
  const int64_t base = bwd ? a.b_off2[layer] : a.f_off[layer];
  const bool head = layer == a.n_layers - 1;
  const int64_t total = (int64_t)ot * ks * 64;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(e % 64);
    const int s = (int)((e / 64) % ks);
    const int t = (int)(e / (64 * (int64_t)ks));
    const int row = 32 * t + (l % 32), g = l / 32;
    float v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      int o, i;  // W[o][i]
      if (!bwd) {
        o = row;
        i = layer == 0 ? fk_natural(s, g, m) : fk_chained(s, g, m);
      } else {
        i = row;
        o = head ? fk_natural(s, g, m) : fk_chained(s, g, m);
      }
      v[m] = (o < out && i < in) ? w[(int64_t)o * in + i] : 0.0f;
    }
    a.pack[base + e] = fpack8(v);
  }
  if (!bwd) {
    const int nb = ot * 32;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x)
      a.bias[a.bias_off[layer] + i] = i < out ? a.w[a.b_off[layer] + i] : 0.0f;
  }
}

// ----------------------------------------------------------------------------- forward
struct FwdArgs {
  const float* grid;
  const int* stats;           // QAT (s, z) per level, or null
  const int32_t* ids;
  int64_t n, n_positions;
  int n_levels, base_res, F, blocks_w, blocks_h, in_dim;
  int shift_x, shift_y;       // pow2_shift of the block grid, -1: the division path
  int64_t level_offset[NTBC_MAX_LEVELS + 1];
  const u32x4* wpack;
  const float* bias;
  int bias_off[kFMaxLayers];
  int n_layers, head_dim, n_bias;
  int64_t bpad;               // positions of the slice-major buffers (a multiple of kSlice)
  uint16_t* xt;               // layer-0 inputs, 16*KS0 rows, bfloat16, slice-major
  uint16_t* ht;               // hidden outputs (after the ReLU), n_hidden regions of HID rows, bfloat16, slice-major
  uint32_t* masks;            // per wave tile and hidden layer: HID/64 words a lane (ReLU derivative bits)
  float* y;                   // [n][y_ld] sigmoid heads
  int y_ld;
  FChunks ct;
};

// Features c0 .. c0+7 of a position (the layer-0 B operand values), from the FP32 master grid
// fake-quantised per level when QAT is on: the arithmetic of k_features.
__device__ __forceinline__ void ffeatures(const FwdArgs& a, int c0, int bx, int by, float v[8]) {
#pragma unroll
  for (int m = 0; m < 8; ++m) v[m] = 0.0f;
  if (a.F == 8) {
    if (c0 >= a.in_dim) return;
    const int l = c0 / 8;
    const int res = a.base_res << l;
    const dev::Corner cx = a.shift_x >= 0 ? dev::corner_pow2(bx, a.blocks_w, res, a.shift_x) : dev::corner(bx, a.blocks_w, res);
    const dev::Corner cy = a.shift_y >= 0 ? dev::corner_pow2(by, a.blocks_h, res, a.shift_y) : dev::corner(by, a.blocks_h, res);
    const int64_t v00 = a.level_offset[l] + (int64_t)cy.i0 * res + cx.i0;
    const int64_t vtx[4] = {v00, v00 + 1, v00 + res, v00 + res + 1};
    const float w[4] = {(1.0f - cx.f) * (1.0f - cy.f), cx.f * (1.0f - cy.f), (1.0f - cx.f) * cy.f, cx.f * cy.f};
    float q[4][8];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float4 lo = *reinterpret_cast<const float4*>(a.grid + vtx[c] * 8);
      const float4 hi = *reinterpret_cast<const float4*>(a.grid + vtx[c] * 8 + 4);
      q[c][0] = lo.x, q[c][1] = lo.y, q[c][2] = lo.z, q[c][3] = lo.w;
      q[c][4] = hi.x, q[c][5] = hi.y, q[c][6] = hi.z, q[c][7] = hi.w;
    }
    if (a.stats) {
      const float s = reinterpret_cast<const float*>(a.stats)[2 * NTBC_MAX_LEVELS + l];
      const int z = a.stats[3 * NTBC_MAX_LEVELS + l];
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          bool inside;
          q[c][m] = fake_quant(q[c][m], s, z, &inside);
        }
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = fmaf(w[0], q[0][m], fmaf(w[1], q[1][m], fmaf(w[2], q[2][m], w[3] * q[3][m])));
    return;
  }
  for (int m = 0; m < 8; ++m) {
    const int c = c0 + m;
    if (c >= a.in_dim) break;
    const int l = c / a.F, f = c % a.F;
    const int res = a.base_res << l;
    const dev::Corner cx = a.shift_x >= 0 ? dev::corner_pow2(bx, a.blocks_w, res, a.shift_x) : dev::corner(bx, a.blocks_w, res);
    const dev::Corner cy = a.shift_y >= 0 ? dev::corner_pow2(by, a.blocks_h, res, a.shift_y) : dev::corner(by, a.blocks_h, res);
    const int64_t v00 = a.level_offset[l] + (int64_t)cy.i0 * res + cx.i0;
    const int64_t vtx[4] = {v00, v00 + 1, v00 + res, v00 + res + 1};
    const float w[4] = {(1.0f - cx.f) * (1.0f - cy.f), cx.f * (1.0f - cy.f), (1.0f - cx.f) * cy.f, cx.f * cy.f};
    float q[4];
    for (int k = 0; k < 4; ++k) {
      q[k] = a.grid[vtx[k] * a.F + f];
      if (a.stats) {
        bool inside;
        q[k] = fake_quant(q[k], reinterpret_cast<const float*>(a.stats)[2 * NTBC_MAX_LEVELS + l],
                          a.stats[3 * NTBC_MAX_LEVELS + l], &inside);
      }
    }
    v[m] = fmaf(w[0], q[0], fmaf(w[1], q[1], fmaf(w[2], q[2], w[3] * q[3])));
  }
}

// Bias-initialised accumulators of output tile t (bias4[q] = neurons 32t + 8q + 4g .. +3).
__device__ __forceinline__ f32x16_t facc_bias(const float* bt, int g) {
  f32x16_t r;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 b = *reinterpret_cast<const float4*>(bt + 8 * q + 4 * g);
    r[4 * q] = b.x, r[4 * q + 1] = b.y, r[4 * q + 2] = b.z, r[4 * q + 3] = b.w;
  }
  return r;
}

// The weight gradient's operands (layer inputs and dZ, bfloat16) are stored slice-major: a region of
// `rows` rows over bpad positions holds element (r, p) at ((p / kSlice) rows + r) kSlice + p % kSlice,
// so one K slice of the weight-gradient product (all rows, kSlice positions) is one contiguous range.
// The stores (32 rows x the wave's 32 positions at a time) go through a per-wave LDS patch: each lane
// writes its values of the 32 rows at its position (two-byte LDS writes), then lane l reads row l/2,
// positions 16(l%2) .. +15 and stores them as two 16-byte words.  A wave's LDS operations complete in issue order, so
// the wave needs no barrier between its writes and its reads, nor before its next patch.
constexpr int kSlice = 64;                           // positions per slice of the slice-major layout
constexpr int kPatchLd = 40;                         // bfloat16 per patch row (80 bytes: the two lane
                                                     // groups' rows fall on different LDS banks)
constexpr int kPatchBytes = 32 * kPatchLd * 2;       // per wave
static_assert(kPatchBytes % 16 == 0, "patch alignment");

struct FStore {
  uint16_t* patch;  // the wave's LDS patch
  int j, lane;
  int64_t p0;       // the wave's first position (a multiple of 32)
};

__device__ __forceinline__ uint16_t fhalf(const uint32_t* w, int v) { return (uint16_t)((w[v / 2] >> (16 * (v % 2))) & 0xFFFFu); }

// Reads the patch back and stores rows row0 .. row0+31 (those below n_rows) of the slice-major region
// buf of `rows` rows.
__device__ __forceinline__ void fpatch_out(const FStore& st, uint16_t* __restrict__ buf, int rows, int row0,
                                           int n_rows) {
  const int row = st.lane >> 1, h = st.lane & 1;
  const u32x4 lo = *reinterpret_cast<const u32x4*>(st.patch + row * kPatchLd + 16 * h);
  const u32x4 hi = *reinterpret_cast<const u32x4*>(st.patch + row * kPatchLd + 16 * h + 8);
  if (row0 + row < n_rows) {
    int nr = rows;
    asm volatile("" : "+s"(nr));
    const uint32_t slice = (uint32_t)(st.p0 / kSlice);
    uint16_t* dst = buf + (slice * (uint32_t)nr + (uint32_t)(row0 + row)) * (uint32_t)kSlice +
                    (uint32_t)(st.p0 % kSlice) + 16 * h;
    *reinterpret_cast<u32x4*>(dst) = lo;
    *reinterpret_cast<u32x4*>(dst + 8) = hi;
  }
}

// Two 16-row K-step operands (rows 32 pair + 16 u + 8g + m, m < 8, of operand x[u]) stored at the
// lane's position: rows at or past n_rows are not stored.
__device__ __forceinline__ void fstore_ksteps(const FStore& st, uint16_t* __restrict__ buf, int rows, int pair, int g,
                                              const u32x4& x0, const u32x4& x1, int n_rows) {
  const uint32_t w0[4] = {x0[0], x0[1], x0[2], x0[3]}, w1[4] = {x1[0], x1[1], x1[2], x1[3]};
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    st.patch[(8 * g + m) * kPatchLd + st.j] = fhalf(w0, m);
    st.patch[(16 + 8 * g + m) * kPatchLd + st.j] = fhalf(w1, m);
  }
  fpatch_out(st, buf, rows, 32 * pair, n_rows);
}

// The 16 bfloat16 values of an epilogue tile (words w: value v in the half v%2 of word v/2; value v is
// neuron 32t + 8(v/4) + 4g + v%4), zero for positions past the batch.
__device__ __forceinline__ void fstore_tile(const FStore& st, uint16_t* __restrict__ buf, int rows, int t, int g,
                                            const uint32_t (&w)[8], bool live) {
#pragma unroll
  for (int v = 0; v < 16; ++v)
    st.patch[(8 * (v / 4) + 4 * g + v % 4) * kPatchLd + st.j] = live ? fhalf(w, v) : (uint16_t)0;
  fpatch_out(st, buf, rows, 32 * t, rows);
}

// Forward epilogue of a hidden tile: ReLU (NaN kept, so a non-finite parameter reaches the gradient
// check), the next product's two B operands, the derivative bits (z > 0) and the bfloat16 outputs
// stored position-contiguous (zero for positions past the batch).
__device__ __forceinline__ uint32_t fhidden_epilogue(const f32x16_t& acc, int t, int g, u32x4* lo, u32x4* hi,
                                                     uint16_t* __restrict__ ht, int rows, const FStore& st,
                                                     bool live) {
  float r[16];
  uint32_t bits = 0;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const float z = acc[v];
    r[v] = z < 0.0f ? 0.0f : z;
    bits |= (z > 0.0f ? 1u : 0u) << v;
  }
  *lo = fpack8(r);
  *hi = fpack8(r + 8);
  const uint32_t w[8] = {(*lo)[0], (*lo)[1], (*lo)[2], (*lo)[3], (*hi)[0], (*hi)[1], (*hi)[2], (*hi)[3]};
  fstore_tile(st, ht, rows, t, g, w, live);
  return bits;
}

template <int S, int T>
__device__ __forceinline__ void fwd_hidden(const FwdArgs& a, const u32x4 (&in)[S], u32x4 (&out)[S], const float* bl,
                                           uint16_t* __restrict__ ht, uint32_t* __restrict__ mk, u32x4* smem, int& c,
                                           int tid, int lane, int g, const FStore& st, bool live) {
#pragma unroll
  for (int tc = 0; tc < T / kFChunkTiles; ++tc) {
    fchunk_dma(a.wpack, a.ct, c + 1, smem + ((c + 1) & 1) * a.ct.cap, tid);
    f32x16_t acc[kFChunkTiles];
#pragma unroll
    for (int u = 0; u < kFChunkTiles; ++u) acc[u] = facc_bias(bl + 32 * (kFChunkTiles * tc + u), g);
    fchunk_mfma<S, S>(smem + (c & 1) * a.ct.cap, in, lane, kFChunkTiles, acc);
    uint32_t word = 0;
#pragma unroll
    for (int u = 0; u < kFChunkTiles; ++u) {
      const int t = kFChunkTiles * tc + u;
      word |= fhidden_epilogue(acc[u], t, g, &out[2 * t], &out[2 * t + 1], ht, 32 * T, st, live) << (16 * u);
    }
    mk[tc * 64] = word;
    fwait_dma();
    __syncthreads();
    ++c;
  }
}

template <int HID, int KS0, int NH, int HT>
__global__ void __launch_bounds__(64 * kFW) __attribute__((amdgpu_waves_per_eu(2))) k_train_fwd(FwdArgs a) {
  constexpr int S = HID / 16, T = HID / 32;
  extern __shared__ u32x4 smem[];
  float* bias_s = reinterpret_cast<float*>(smem + 2 * a.ct.cap + kFW * kPatchBytes / 16);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, j = lane & 31, g = lane >> 5;
  const int64_t p = (int64_t)blockIdx.x * kFPos + wave * 32 + j;
  const bool live = p < a.n;
  const FStore st{reinterpret_cast<uint16_t*>(smem + 2 * a.ct.cap + wave * kPatchBytes / 16), j, lane, p - j};
  const int id = live ? clamp_id(a.ids[p], a.n_positions) : 0;
  const int bx = id % a.blocks_w, by = id / a.blocks_w;
  const int n_hidden = a.n_layers - 1;
  uint32_t* mbase = a.masks + ((int64_t)(blockIdx.x * kFW + wave) * n_hidden) * (T / 2) * 64 + lane;

  fchunk_dma(a.wpack, a.ct, 0, smem, tid);
  for (int i = tid; i < a.n_bias; i += 64 * kFW) bias_s[i] = a.bias[i];
  u32x4 x0[KS0];
#pragma unroll
  for (int s = 0; s < KS0; ++s) {
    float v[8];
    ffeatures(a, 16 * s + 8 * g, bx, by, v);
    if (!live) {
#pragma unroll
      for (int m = 0; m < 8; ++m) v[m] = 0.0f;
    }
    x0[s] = fpack8(v);
  }
#pragma unroll
  for (int s = 0; s < KS0; s += 2) fstore_ksteps(st, a.xt, 16 * KS0, s / 2, g, x0[s], s + 1 < KS0 ? x0[s + 1] : u32x4{}, 16 * KS0);
  fwait_dma();
  __syncthreads();

  int c = 0;
  u32x4 bin[S], bout[S];
  {
    const float* bl = bias_s + a.bias_off[0];
    uint32_t* mk = mbase;
#pragma unroll
    for (int tc = 0; tc < T / kFChunkTiles; ++tc) {
      fchunk_dma(a.wpack, a.ct, c + 1, smem + ((c + 1) & 1) * a.ct.cap, tid);
      f32x16_t acc[kFChunkTiles];
#pragma unroll
      for (int u = 0; u < kFChunkTiles; ++u) acc[u] = facc_bias(bl + 32 * (kFChunkTiles * tc + u), g);
      fchunk_mfma<KS0, KS0>(smem + (c & 1) * a.ct.cap, x0, lane, kFChunkTiles, acc);
      uint32_t word = 0;
#pragma unroll
      for (int u = 0; u < kFChunkTiles; ++u) {
        const int t = kFChunkTiles * tc + u;
        word |= fhidden_epilogue(acc[u], t, g, &bin[2 * t], &bin[2 * t + 1], a.ht, HID, st, live) << (16 * u);
      }
      mk[tc * 64] = word;
      fwait_dma();
      __syncthreads();
      ++c;
    }
  }
  static_assert(NH >= 1 && NH <= 2, "one or two middle hidden layers");
  fwd_hidden<S, T>(a, bin, bout, bias_s + a.bias_off[1], a.ht + (int64_t)HID * a.bpad, mbase + (T / 2) * 64, smem, c, tid,
                   lane, g, st, live);
  if constexpr (NH == 2) {
    fwd_hidden<S, T>(a, bout, bin, bias_s + a.bias_off[2], a.ht + (int64_t)2 * HID * a.bpad, mbase + 2 * (T / 2) * 64,
                     smem, c, tid, lane, g, st, live);
  } else {
#pragma unroll
    for (int s = 0; s < S; ++s) bin[s] = bout[s];
  }
  // head: sigmoid outputs in rows 32t + 8q + 4g .. +3 of position p
  const float* bl = bias_s + a.bias_off[NH + 1];
#pragma unroll
  for (int tc = 0; tc < (HT + 1) / 2; ++tc) {
    fchunk_dma(a.wpack, a.ct, c + 1, smem + ((c + 1) & 1) * a.ct.cap, tid);
    const int valid = HT - kFChunkTiles * tc < kFChunkTiles ? HT - kFChunkTiles * tc : kFChunkTiles;
    f32x16_t acc[kFChunkTiles];
#pragma unroll
    for (int u = 0; u < kFChunkTiles; ++u) acc[u] = u < valid ? facc_bias(bl + 32 * (kFChunkTiles * tc + u), g) : f32x16_t{};
    fchunk_mfma<S, S>(smem + (c & 1) * a.ct.cap, bin, lane, valid, acc);
#pragma unroll
    for (int u = 0; u < kFChunkTiles; ++u) {
      if (u < valid && live) {
        const int t = kFChunkTiles * tc + u;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r0 = 32 * t + 8 * q + 4 * g;
          float o[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) o[r] = fsigmoid(acc[u][4 * q + r]);
          float* dst = a.y + p * a.y_ld + r0;
          if ((a.y_ld & 3) == 0) {
            if (r0 < a.head_dim) *reinterpret_cast<float4*>(dst) = float4{o[0], o[1], o[2], o[3]};
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (r0 + r < a.head_dim) dst[r] = o[r];
          }
        }
      }
    }
    fwait_dma();
    __syncthreads();
    ++c;
  }
}

// ----------------------------------------------------------------------------- backward
struct BwdArgs {
  const float* dz;            // [n][dz_ld] dL/dZ of the head pre-activations
  int dz_ld, head_dim;
  int64_t n, bpad;
  const u32x4* wpack;
  const uint32_t* masks;
  uint16_t* dzt;              // bfloat16 dZ_k, slice-major: layer k's region (out_pad rows) starts at row zrow[k]
  int64_t zrow[kFMaxLayers];
  float* dx;                  // [n][in_dim]
  int in_dim, n_layers;
  FChunks ct;
};

// Backward epilogue of a tile: dZ = dH * (z > 0) (`bits`), the next product's B operands, and the
// bfloat16 dZ stored position-contiguous.
__device__ __forceinline__ void fbwd_epilogue(const f32x16_t& acc, uint32_t bits, int t, int g, u32x4* lo, u32x4* hi,
                                              uint16_t* __restrict__ zt, int rows, const FStore& st, bool live) {
  float r[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) r[v] = ((bits >> v) & 1u) ? acc[v] : 0.0f;
  *lo = fpack8(r);
  *hi = fpack8(r + 8);
  const uint32_t w[8] = {(*lo)[0], (*lo)[1], (*lo)[2], (*lo)[3], (*hi)[0], (*hi)[1], (*hi)[2], (*hi)[3]};
  fstore_tile(st, zt, rows, t, g, w, live);
}

// One backward product W_k^T dZ_k over a hidden layer's rows (T tiles), K = KS steps of `in`.
template <int KS, int NB, int S, int T>
__device__ __forceinline__ void bwd_hidden(const BwdArgs& a, const u32x4 (&in)[NB], u32x4 (&out)[S],
                                           const uint32_t* __restrict__ mk, uint16_t* __restrict__ zt, u32x4* smem,
                                           int& c, int tid, int lane, int g, const FStore& st, bool live) {
#pragma unroll
  for (int tc = 0; tc < T / kFChunkTiles; ++tc) {
    fchunk_dma(a.wpack, a.ct, c + 1, smem + ((c + 1) & 1) * a.ct.cap, tid);
    f32x16_t acc[kFChunkTiles];
#pragma unroll
    for (int u = 0; u < kFChunkTiles; ++u) acc[u] = f32x16_t{};
    fchunk_mfma<KS, NB>(smem + (c & 1) * a.ct.cap, in, lane, kFChunkTiles, acc);
    const uint32_t word = mk[tc * 64];
#pragma unroll
    for (int u = 0; u < kFChunkTiles; ++u) {
      const int t = kFChunkTiles * tc + u;
      fbwd_epilogue(acc[u], word >> (16 * u), t, g, &out[2 * t], &out[2 * t + 1], zt, 32 * T, st, live);
    }
    fwait_dma();
    __syncthreads();
    ++c;
  }
}

template <int HID, int KS0, int NH, int HT>
__global__ void __launch_bounds__(64 * kFW) __attribute__((amdgpu_waves_per_eu(2))) k_train_bwd(BwdArgs a) {
  constexpr int S = HID / 16, T = HID / 32;
  constexpr int KH = 2 * HT;        // K-steps of the head gradient
  constexpr int IT = (KS0 + 1) / 2; // row tiles of dX
  extern __shared__ u32x4 smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, j = lane & 31, g = lane >> 5;
  const int64_t p = (int64_t)blockIdx.x * kFPos + wave * 32 + j;
  const bool live = p < a.n;
  const FStore st{reinterpret_cast<uint16_t*>(smem + 2 * a.ct.cap + wave * kPatchBytes / 16), j, lane, p - j};
  const int n_hidden = a.n_layers - 1;
  const uint32_t* mbase = a.masks + ((int64_t)(blockIdx.x * kFW + wave) * n_hidden) * (T / 2) * 64 + lane;

  fchunk_dma(a.wpack, a.ct, 0, smem, tid);
  // head gradient: B operands in natural row order, also stored position-contiguous for dW
  u32x4 dzh[KH];
  uint16_t* zh = a.dzt + a.zrow[a.n_layers - 1] * a.bpad;
#pragma unroll
  for (int s = 0; s < KH; ++s) {
    float v[8];
    const int r0 = 16 * s + 8 * g;
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = (live && r0 + m < a.head_dim) ? a.dz[p * a.dz_ld + r0 + m] : 0.0f;
    dzh[s] = fpack8(v);
  }
#pragma unroll
  for (int s = 0; s < KH; s += 2) fstore_ksteps(st, zh, 16 * KH, s / 2, g, dzh[s], dzh[s + 1], 16 * KH);
  fwait_dma();
  __syncthreads();

  int c = 0;
  u32x4 bin[S], bout[S];
  const int top = a.n_layers - 2;  // the last hidden layer
  // head^T: dZ of the last hidden layer
  bwd_hidden<KH, KH, S, T>(a, dzh, bin, mbase + top * (T / 2) * 64, a.dzt + a.zrow[top] * a.bpad, smem, c, tid, lane, g,
                           st, live);
  // middle layers, from the top down
  static_assert(NH >= 1 && NH <= 2, "one or two middle hidden layers");
  bwd_hidden<S, S, S, T>(a, bin, bout, mbase + (top - 1) * (T / 2) * 64, a.dzt + a.zrow[top - 1] * a.bpad, smem, c,
                         tid, lane, g, st, live);
  if constexpr (NH == 2) {
    bwd_hidden<S, S, S, T>(a, bout, bin, mbase + (top - 2) * (T / 2) * 64, a.dzt + a.zrow[top - 2] * a.bpad, smem, c,
                           tid, lane, g, st, live);
  } else {
#pragma unroll
    for (int s = 0; s < S; ++s) bin[s] = bout[s];
  }
  // dX = W_0^T dZ_0 in FP32: features 32t + 8q + 4g .. +3 of position p
#pragma unroll
  for (int tc = 0; tc < (IT + 1) / 2; ++tc) {
    fchunk_dma(a.wpack, a.ct, c + 1, smem + ((c + 1) & 1) * a.ct.cap, tid);
    const int valid = IT - kFChunkTiles * tc < kFChunkTiles ? IT - kFChunkTiles * tc : kFChunkTiles;
    f32x16_t acc[kFChunkTiles];
#pragma unroll
    for (int u = 0; u < kFChunkTiles; ++u) acc[u] = f32x16_t{};
    fchunk_mfma<S, S>(smem + (c & 1) * a.ct.cap, bin, lane, valid, acc);
    if (live) {
#pragma unroll
      for (int u = 0; u < kFChunkTiles; ++u) {
        if (u < valid) {
          const int t = kFChunkTiles * tc + u;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int f0 = 32 * t + 8 * q + 4 * g;
            float* dst = a.dx + p * a.in_dim + f0;
            if ((a.in_dim & 3) == 0) {
              if (f0 < a.in_dim)
                *reinterpret_cast<float4*>(dst) = float4{acc[u][4 * q], acc[u][4 * q + 1], acc[u][4 * q + 2], acc[u][4 * q + 3]};
            } else {
#pragma unroll
              for (int r = 0; r < 4; ++r)
                if (f0 + r < a.in_dim) dst[r] = acc[u][4 * q + r];
            }
          }
        }
      }
    }
    fwait_dma();
    __syncthreads();
    ++c;
  }
}

// ----------------------------------------------------------------------------- weight gradient
struct DwJob {
  const uint16_t* a;  // A(m, k): dZ_k rows (output neurons), slice-major region of a_rows rows
  const uint16_t* b;  // B(n, k): layer inputs, slice-major region of b_rows rows
  int a_rows, b_rows; // rows present in the buffers (padded, zero past the true sizes)
  int M, N;           // true output sizes
  int tiles_n, tile0; // 128-wide tiles along N; first global tile of the job
  float* c;           // dW [M][N] (canonical row-major)
  float* db;          // bias gradient [M]
};

struct DwArgs {
  DwJob job[kFMaxLayers];
  int n_jobs, n_tiles, splits, k_split;
  int64_t bpad, K;    // K = positions (a multiple of 32)
  float* part;        // [n_tiles][splits][128 * 128]
  float* dbpart;      // [n_tiles][splits][128]
  int assign;         // write the sums to dW and db instead of adding them
  float* flag;        // when set: *flag = 1 if any dW or db element written is not finite
};

// Block b: tile b % n_tiles, K range b / n_tiles.  Four waves, each a 64 x 64 quadrant as 2 x 2
// products of 32 x 32.  The K range advances in slices of kDwK positions: each thread loads kDwK/16
// x 16 bytes of A rows and of B rows (row tid/2, positions (kDwK/2)(tid%2) .. +kDwK/2-1 of the slice)
// into registers while the previous slice is multiplied from LDS, then stores them to the other LDS
// buffer (one barrier per slice); a lane's fragment (row l%32, positions 8(l/32) .. +7 of a K-step) is
// one 16-byte LDS read.
constexpr int kDwK = kSlice;      // positions per slice (one slice of the slice-major operands)
constexpr int kDwRow = kDwK + 8;  // LDS row stride in bfloat16 (144 bytes)
constexpr int kDwLd = kDwK / 16;  // 16-byte loads per thread and operand

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_train_dw(DwArgs a) {
  __shared__ __align__(16) uint16_t As[2][128][kDwRow];
  __shared__ __align__(16) uint16_t Bs[2][128][kDwRow];
  // Workgroups are dispatched round-robin over the eight XCDs; give each XCD a contiguous run of
  // (split, tile) pairs, tiles fastest, so the tiles that read the same K range of the same A (or B)
  // rows run at the same time on one XCD and the second read hits its L2.
  const int nwg = (int)gridDim.x, per = nwg / 8, extra = nwg % 8, x = (int)blockIdx.x % 8, kx = (int)blockIdx.x / 8;
  const int flat = x * per + (x < extra ? x : extra) + kx;
  const int tile = flat % a.n_tiles, split = flat / a.n_tiles;
  int jb = 0;
  while (jb + 1 < a.n_jobs && tile >= a.job[jb + 1].tile0) ++jb;
  const DwJob& J = a.job[jb];
  const int lt = tile - J.tile0;
  const int tm = lt / J.tiles_n, tn = lt % J.tiles_n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1, li = lane & 31, g = lane >> 5;
  const int64_t k0 = (int64_t)split * a.k_split;
  const int64_t k1 = k0 + a.k_split < a.K ? k0 + a.k_split : a.K;
  // the thread's staging row and half slice
  const int sr = tid >> 1, sh = (tid & 1) * (kDwK / 2);
  const int arow = tm * 128 + sr, brow = tn * 128 + sr;
  const bool aok = arow < J.a_rows, bok = brow < J.b_rows;
  // slice-major operands: slice k / kDwK of a region starts (k / kDwK) rows kDwK elements in
  const uint16_t* ag = J.a + (int64_t)(aok ? arow : 0) * kDwK + sh;
  const uint16_t* bg = J.b + (int64_t)(bok ? brow : 0) * kDwK + sh;
  const int64_t astep = (int64_t)J.a_rows * kDwK, bstep = (int64_t)J.b_rows * kDwK;
  const bool sums = tn == 0;  // bias gradient: row sums of A in FP32
  float rs = 0.0f;
  // two register stages, so that two slices are in flight while one is multiplied; the loop below runs
  // in pairs of slices so that every stage index is a compile-time constant
  u32x4 ra[2][kDwLd], rb[2][kDwLd];
  auto load = [&](int64_t k, int r) {
    const u32x4* ap = reinterpret_cast<const u32x4*>(ag + (k / kDwK) * astep);
    const u32x4* bp = reinterpret_cast<const u32x4*>(bg + (k / kDwK) * bstep);
#pragma unroll
    for (int h = 0; h < kDwLd; ++h) {
      ra[r][h] = aok ? ap[h] : u32x4{};
      rb[r][h] = bok ? bp[h] : u32x4{};
    }
  };
  // the row sums are taken here, when the slice is needed anyway, not at the load (which would wait)
  auto store = [&](int r, int buf) {
    if (sums) {
#pragma unroll
      for (int h = 0; h < kDwLd; ++h)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          rs += __uint_as_float(ra[r][h][e] << 16) + __uint_as_float(ra[r][h][e] & 0xFFFF0000u);
    }
#pragma unroll
    for (int h = 0; h < kDwLd; ++h) {
      *reinterpret_cast<u32x4*>(&As[buf][sr][sh + 8 * h]) = ra[r][h];
      *reinterpret_cast<u32x4*>(&Bs[buf][sr][sh + 8 * h]) = rb[r][h];
    }
  };
  f32x16_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) acc[i][jj] = f32x16_t{};
  auto mult = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < kDwK / 16; ++ks) {
      u32x4 af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        af[i] = *reinterpret_cast<const u32x4*>(&As[buf][wm * 64 + 32 * i + li][16 * ks + 8 * g]);
        bf[i] = *reinterpret_cast<const u32x4*>(&Bs[buf][wn * 64 + 32 * i + li][16 * ks + 8 * g]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) acc[i][jj] = fmma(af[i], bf[jj], acc[i][jj]);
    }
  };
  // slice k lives in LDS buffer (k - k0) / kDwK % 2; register stage 0 carries the even slices, 1 the odd
  if (k0 < k1) {
    load(k0, 0);
    if (k0 + kDwK < k1) load(k0 + kDwK, 1);
    store(0, 0);
  }
  __syncthreads();
  for (int64_t k = k0; k < k1; k += 2 * kDwK) {
    // even slice k from buffer 0; slice k + kDwK arrives in stage 1, slice k + 2 kDwK is fetched into stage 0
    if (k + 2 * kDwK < k1) load(k + 2 * kDwK, 0);
    mult(0);
    if (k + kDwK < k1) store(1, 1);
    __syncthreads();
    if (k + kDwK >= k1) break;
    // odd slice k + kDwK from buffer 1; slice k + 2 kDwK arrives in stage 0, k + 3 kDwK is fetched into stage 1
    if (k + 3 * kDwK < k1) load(k + 3 * kDwK, 1);
    mult(1);
    if (k + 2 * kDwK < k1) store(0, 0);
    __syncthreads();
  }
  float* part = a.part + ((int64_t)tile * a.splits + split) * (128 * 128);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = wm * 64 + 32 * i + 8 * (v / 4) + 4 * g + v % 4;
        const int col = wn * 64 + 32 * jj + li;
        part[r * 128 + col] = acc[i][jj][v];
      }
  if (sums) {
    const float t = rs + __shfl_xor(rs, 1);  // the two threads of a staging row
    if ((tid & 1) == 0) a.dbpart[((int64_t)tile * a.splits + split) * 128 + sr] = t;
  }
}

// dW (and db) += the sum of the partial tiles over the K ranges, in K-range order (= with a.assign); one
// thread per element of a tile.
__global__ void __launch_bounds__(256) k_train_dw_reduce(DwArgs a) {
  const int tile = blockIdx.y;
  int jb = 0;
  while (jb + 1 < a.n_jobs && tile >= a.job[jb + 1].tile0) ++jb;
  const DwJob& J = a.job[jb];
  const int lt = tile - J.tile0;
  const int tm = lt / J.tiles_n, tn = lt % J.tiles_n;
  const float* part = a.part + (int64_t)tile * a.splits * (128 * 128);
  const int e = blockIdx.x * 256 + threadIdx.x;  // gridDim.x = 64
  const int r = e / 128, col = e % 128;
  const int m = tm * 128 + r, nn = tn * 128 + col;
  bool bad = false;
  if (m < J.M && nn < J.N) {
    float s = 0.0f;
    // unrolled so that eight loads are in flight; the additions stay in split order
#pragma unroll 8
    for (int k = 0; k < a.splits; ++k) s += part[(int64_t)k * (128 * 128) + e];
    float* dst = J.c + (int64_t)m * J.N + nn;
    const float v = a.assign ? s : *dst + s;
    *dst = v;
    bad = !isfinite(v);
  }
  if (tn == 0 && blockIdx.x == 0 && threadIdx.x < 128) {
    const int mr = tm * 128 + threadIdx.x;
    if (mr < J.M) {
      float s = 0.0f;
#pragma unroll 8
      for (int k = 0; k < a.splits; ++k) s += a.dbpart[((int64_t)tile * a.splits + k) * 128 + threadIdx.x];
      const float v = a.assign ? s : J.db[mr] + s;
      J.db[mr] = v;
      bad |= !isfinite(v);
    }
  }
  if (a.flag != nullptr && __ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicExch(a.flag, 1.0f);
}

// ------------------------------------------------------------------------------------------ batches
__host__ __device__ __forceinline__ uint64_t splitmix_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__global__ void k_batch_ids(uint64_t key, int32_t batch, uint64_t n_positions, int32_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  const uint64_t z = splitmix_out(key + (uint64_t)(i + 1) * kGamma);
  out[i] = (int32_t)(((z >> 32) * n_positions) >> 32);
}

// ------------------------------------------------------------------------------------------ host
int fill(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return NTBC_OK;
  const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(ceil_div(n, 4), 256), 4096);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, p, n, v);
  return check_launch("k_fill");
}

LevelArgs level_args(const Shape& s) {
  LevelArgs la{};
  la.n_levels = s.n_levels;
  for (int l = 0; l < s.n_levels; ++l) {
    la.begin[l] = s.level_offset[l] * s.n_features;
    la.count[l] = (s.level_offset[l + 1] - s.level_offset[l]) * s.n_features;
  }
  return la;
}

int qat_range(const Shape& s, const float* grid, int* stats, hipStream_t strm) {
  hipLaunchKernelGGL(k_init_stats, dim3(1), dim3(64), 0, strm, stats);
  MinMaxArgs ma{};
  ma.g = grid;
  ma.n_levels = s.n_levels;
  int blocks = 0;
  for (int l = 0; l < s.n_levels; ++l) {
    ma.begin[l] = s.level_offset[l] * s.n_features;
    ma.count[l] = (s.level_offset[l + 1] - s.level_offset[l]) * s.n_features;
    ma.first_block[l] = blocks;
    blocks += (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(ma.count[l], 8 * kBlock), 2048));
  }
  ma.first_block[s.n_levels] = blocks;
  hipLaunchKernelGGL(k_level_minmax, dim3(blocks), dim3(kBlock), 0, strm, ma, stats);
  hipLaunchKernelGGL(k_qat_params, dim3(1), dim3(64), 0, strm, stats, s.n_levels);
  return check_launch("qat range");
}

FeatArgs feat_args(const Shape& s, const float* grid, const int* stats, const int32_t* ids, int64_t n, float* x) {
  FeatArgs f{};
  f.grid = grid;
  f.stats = stats;
  f.ids = ids;
  f.n = n;
  f.n_levels = s.n_levels;
  f.base_res = s.base_res;
  f.F = s.n_features;
  f.blocks_w = s.blocks_w;
  f.blocks_h = s.blocks_h;
  f.shift_x = pow2_shift(s, s.blocks_w);
  f.shift_y = pow2_shift(s, s.blocks_h);
  for (int l = 0; l <= s.n_levels; ++l) f.level_offset[l] = s.level_offset[l];
  f.x = x;
  return f;
}

struct Ctx {
  Shape s;
  TrainLayout lay;
  float* ws;
  int64_t n;
  hipStream_t strm;
  bool bf16;  // bfloat16 matrix-core operands (FP32 accumulation, FP32 master parameters)
  bool det = false;     // deterministic reductions (grid scatter in fixed point, unsplit weight products)
  bool selu = false;    // SELU hidden layers (the paper's own layout) instead of ReLU
  bool texel_blocks = false;  // the positions are the 16 texels of each block in turn (texel-grid ids)
  int64_t det_off = 0;  // byte offset of the deterministic scatter's sums in the workspace
  int* stats() { return reinterpret_cast<int*>(ws + lay.stats); }
  float* act_in(int k) { return k == 0 ? ws + lay.x : ws + lay.h[k - 1]; }
};

int64_t det_offset(const Shape& s, int64_t batch);

int check_common(const ntbc_model_desc* d, int precision, const int32_t* ids, int32_t n, void* workspace,
                 size_t workspace_bytes, Ctx* c) {
  int st = make_shape(d, &c->s);
  if (st != NTBC_OK) return st;
  if (precision != NTBC_FP32 && precision != NTBC_BF16)
    return fail(precision == NTBC_FP8_E4M3 || precision == NTBC_FP16 ? NTBC_EUNSUPPORTED : NTBC_EINVAL,
                "training runs in FP32 or BF16 (precision %d)", precision);
  c->bf16 = precision == NTBC_BF16;
  NTBC_REQUIRE(n >= 0, "n %d < 0", n);
  NTBC_REQUIRE(n == 0 || ids != nullptr, "ids is NULL");
  c->lay = train_layout(c->s, n);
  const int64_t need = train_workspace_bytes(c->s, n);
  if (workspace == nullptr || workspace_bytes < (size_t)need)
    return fail(NTBC_ENOWORKSPACE, "workspace needs %lld bytes", (long long)need);
  c->ws = static_cast<float*>(workspace);
  c->n = n;
  c->det_off = det_offset(c->s, n);
  return NTBC_OK;
}

// Forward of the batch: X, hidden activations, heads (into y).
int forward(Ctx& c, const float* grid, const float* weights, bool qat, const int32_t* ids, float* y) {
  const Shape& s = c.s;
  int st;
  if (qat) {
    st = qat_range(s, grid, c.stats(), c.strm);
    if (st != NTBC_OK) return st;
  }
  const FeatArgs fa = feat_args(s, grid, qat ? c.stats() : nullptr, ids, c.n, c.ws + c.lay.x);
  hipLaunchKernelGGL(k_features, dim3((unsigned)ceil_div(c.n * s.n_levels * s.n_features, kBlock)), dim3(kBlock), 0, c.strm, fa);
  st = check_launch("k_features");
  if (st != NTBC_OK) return st;
  for (int k = 0; k < s.n_layers; ++k) {
    GemmArgs g{};
    g.a = c.act_in(k);
    g.sam = s.layer_in[k];
    g.sak = 1;
    g.b = weights + s.w_off[k];
    g.sbk = 1;
    g.sbn = s.layer_in[k];
    const bool last = k == s.n_layers - 1;
    g.c = last ? y : c.ws + c.lay.h[k];
    g.ldc = s.layer_out[k];
    g.M = (int)c.n;
    g.N = s.layer_out[k];
    g.K = s.layer_in[k];
    g.k_split = g.K;
    g.bias = weights + s.b_off[k];
    st = last     ? gemm<EPI_BIAS_SIGMOID>(g, 1, c.strm, c.bf16)
         : c.selu ? gemm<EPI_BIAS_SELU>(g, 1, c.strm, c.bf16)
                  : gemm<EPI_BIAS_RELU>(g, 1, c.strm, c.bf16);
    if (st != NTBC_OK) return st;
  }
  return NTBC_OK;
}

// Grid scatter of dX ([n][in_dim]) into d_grid (QAT pass-through mask when qat).  Deterministic mode:
// 64-bit fixed-point sums at a per-step power-of-two scale (k_det_scale), converted and added at the end.
// Grid levels whose gradient (vbytes a value) fits in kCoarseLds of LDS.
int coarse_levels(const Shape& s, size_t vbytes) {
  int n = 0;
  while (n < s.n_levels && s.level_offset[n + 1] * s.n_features * (int64_t)vbytes <= kCoarseLds) ++n;
  return n;
}

int64_t coarse_offset(const Shape& s, int64_t batch);

// levels: 0 every level, 1 only the LDS-summed coarse levels, 2 only the others (atomic mode only: the
// two parts then touch disjoint vertices and may run on different streams).
int scatter_grid(Ctx& c, const float* grid, bool qat, const int32_t* ids, const float* dx, float* d_grid,
                 int levels = 0) {
  const Shape& s = c.s;
  const FeatArgs fa = feat_args(s, grid, qat ? c.stats() : nullptr, ids, c.n, nullptr);
  const int64_t count = s.grid_vertices * s.n_features;
  char* det = reinterpret_cast<char*>(c.ws) + c.det_off;
  unsigned* amax = reinterpret_cast<unsigned*>(det);
  float* scale = reinterpret_cast<float*>(det + 4);
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(det + 256);
  const size_t vbytes = c.det ? 8 : 4;
  if (c.det) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, c.strm, reinterpret_cast<unsigned long long*>(det), (int64_t)1);
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)std::min<int64_t>(ceil_div(count, 256), 8192)), dim3(256), 0, c.strm, acc, count);
    const int64_t nx = c.n * s.in_dim;
    hipLaunchKernelGGL(k_absmax_bits, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(nx, 256), 1024))), dim3(256), 0,
                       c.strm, dx, nx, amax);
    hipLaunchKernelGGL(k_det_scale, dim3(1), dim3(1), 0, c.strm, amax, c.n, scale);
  }
  // coarse levels whose gradient fits in kCoarseLds of LDS are pre-aggregated per block
  const int n_coarse = coarse_levels(s, vbytes);
  if (n_coarse > 0 && levels != 2) {
    const int64_t nv = s.level_offset[n_coarse] * s.n_features;
    const size_t lds = (size_t)nv * vbytes;
    char* part = reinterpret_cast<char*>(c.ws) + coarse_offset(s, c.n);
    if (c.det) {
      hipLaunchKernelGGL(k_scatter_coarse<unsigned long long>, dim3(kCoarseBlocks), dim3(kCoarseThreads), lds, c.strm, fa, dx,
                         reinterpret_cast<unsigned long long*>(part), n_coarse, (const float*)scale);
      hipLaunchKernelGGL(k_scatter_reduce<unsigned long long>, dim3((unsigned)ceil_div(nv, 64)), dim3(256), 0, c.strm,
                         reinterpret_cast<const unsigned long long*>(part), kCoarseBlocks, nv, acc);
    } else {
      hipLaunchKernelGGL(k_scatter_coarse<float>, dim3(kCoarseBlocks), dim3(kCoarseThreads), lds, c.strm, fa, dx,
                         reinterpret_cast<float*>(part), n_coarse, (const float*)nullptr);
      hipLaunchKernelGGL(k_scatter_reduce<float>, dim3((unsigned)ceil_div(nv, 64)), dim3(256), 0, c.strm,
                         reinterpret_cast<const float*>(part), kCoarseBlocks, nv, d_grid);
    }
  }
  // texel blocks: per-block sums when no fine level is finer than the texel grid
  const int64_t finest = (int64_t)s.base_res << (s.n_levels - 1);
  if (levels == 1) {
    // the fine levels are left to a second call
  } else if (n_coarse < s.n_levels && c.texel_blocks && c.n % 16 == 0 && finest <= s.blocks_w &&
             finest <= s.blocks_h) {
    const dim3 grid_dim((unsigned)ceil_div(c.n / 16 * (s.n_levels - n_coarse) * s.n_features, kBlock));
    if (c.det)
      hipLaunchKernelGGL(k_scatter_texels<unsigned long long>, grid_dim, dim3(kBlock), 0, c.strm, fa, dx, acc, n_coarse,
                         (const float*)scale);
    else
      hipLaunchKernelGGL(k_scatter_texels<float>, grid_dim, dim3(kBlock), 0, c.strm, fa, dx, d_grid, n_coarse,
                         (const float*)nullptr);
  } else if (n_coarse < s.n_levels) {
    const dim3 grid_dim((unsigned)ceil_div(c.n * (s.n_levels - n_coarse) * s.n_features, kBlock));
    if (c.det)
      hipLaunchKernelGGL(k_scatter<unsigned long long>, grid_dim, dim3(kBlock), 0, c.strm, fa, dx, acc, n_coarse,
                         (const float*)scale);
    else
      hipLaunchKernelGGL(k_scatter<float>, grid_dim, dim3(kBlock), 0, c.strm, fa, dx, d_grid, n_coarse, (const float*)nullptr);
  }
  if (c.det)
    hipLaunchKernelGGL(k_det_finish, dim3((unsigned)std::min<int64_t>(ceil_div(count, 256), 8192)), dim3(256), 0, c.strm, acc,
                       (const float*)scale, d_grid, count);
  return check_launch("k_scatter");
}

// Backward of the batch from dZ_out (in lay.dy): accumulates d_weights and d_grid.
int backward(Ctx& c, const float* grid, const float* weights, bool qat, const int32_t* ids, float* d_grid, float* d_weights) {
  const Shape& s = c.s;
  int st;
  float* dz = c.ws + c.lay.dy;
  float* bufs[2] = {c.ws + c.lay.da, c.ws + c.lay.db};
  int nb = 0;
  for (int k = s.n_layers - 1; k >= 0; --k) {
    const int in = s.layer_in[k], out = s.layer_out[k];
    // dW_k += dZ_k^T H_k (split over the batch)
    GemmArgs gw{};
    gw.a = dz;
    gw.sam = 1;
    gw.sak = out;
    gw.b = c.act_in(k);
    gw.sbk = in;
    gw.sbn = 1;
    gw.c = d_weights + s.w_off[k];
    gw.ldc = in;
    gw.M = out;
    gw.N = in;
    gw.K = (int)c.n;
    const int tile = c.bf16 ? kBT : 64;
    const int tiles = (int)(ceil_div(out, tile) * ceil_div(in, tile));
    // split over the batch with atomic adds, or (deterministic mode) one product per output tile
    int splits = c.det ? 1 : (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(c.n, 256), ceil_div(c.bf16 ? 512 : 2048, tiles)));
    const int kq = c.bf16 ? kBTK : 16;
    gw.k_split = (int)(ceil_div(ceil_div(c.n, splits), kq) * kq);
    splits = (int)ceil_div(c.n, gw.k_split);
    // db_k += column sums of dZ_k: fused into the product (the bfloat16 kernel sums A staged MN-contiguous
    // only), a separate kernel otherwise
    const bool fused = !c.bf16 || gw.sak != 1;
    if (fused) gw.colsum = d_weights + s.b_off[k];
    st = gemm<EPI_ATOMIC>(gw, splits, c.strm, c.bf16);
    if (st != NTBC_OK) return st;
    if (!fused) {
      const int rpb = c.det ? (int)c.n : 128;  // deterministic: one block (one atomic add) per column group
      hipLaunchKernelGGL(k_colsum, dim3((unsigned)ceil_div(c.n, rpb), (unsigned)ceil_div(out, 64)), dim3(kBlock), 0,
                         c.strm, dz, c.n, out, rpb, d_weights + s.b_off[k]);
      st = check_launch("k_colsum");
      if (st != NTBC_OK) return st;
    }
    // dH_k = dZ_k W_k, times the activation derivative of the layer input (none for the grid features)
    GemmArgs gd{};
    gd.a = dz;
    gd.sam = out;
    gd.sak = 1;
    gd.b = weights + s.w_off[k];
    gd.sbk = in;
    gd.sbn = 1;
    gd.c = bufs[nb];
    gd.ldc = in;
    gd.M = (int)c.n;
    gd.N = in;
    gd.K = out;
    gd.k_split = out;
    if (k > 0) {
      gd.mask = c.act_in(k);
      gd.ldm = in;
      st = c.selu ? gemm<EPI_SELU_MASK>(gd, 1, c.strm, c.bf16) : gemm<EPI_MASK>(gd, 1, c.strm, c.bf16);
    } else {
      st = gemm<EPI_STORE>(gd, 1, c.strm, c.bf16);
    }
    if (st != NTBC_OK) return st;
    dz = bufs[nb];
    nb ^= 1;
  }
  return scatter_grid(c, grid, qat, ids, dz, d_grid);
}

// dsigmoid: write dL/dZ of the head pre-activations (dL/dY * Y (1 - Y)) instead of dL/dY.
int loss_grad(const Shape& s, const ntbc_targets* t, const float* heads, const int32_t* ids, int64_t n, float temperature,
              const float* lw, float* losses, float* dheads, hipStream_t strm, bool dsigmoid = false, int ld = 0,
              bool losses_zeroed = false) {
  const int st = losses_zeroed ? NTBC_OK : fill(losses, 5, 0.0f, strm);
  if (st != NTBC_OK) return st;
  LossArgs a{};
  a.y = heads;
  a.dy = dheads;
  a.dsigmoid = dsigmoid ? 1 : 0;
  a.ids = ids;
  a.n = n;
  a.n_positions = s.n_positions;
  a.head_dim = s.head_dim;
  a.ld = ld > 0 ? ld : s.head_dim;
  a.E = s.endpoint_dim;
  a.C = s.channels;
  a.n_textures = s.n_textures;
  a.blocks_w = s.blocks_w;
  for (int i = 0; i < s.n_textures; ++i) {
    a.formats[i] = s.formats[i];
    a.ep_off[i] = s.ep_off[i];
    a.ch_off[i] = s.ch_off[i];
    a.tex[i] = t->texels[i];
    a.btex[i] = t->block_texels[i];
  }
  a.blocked = 1;
  for (int i = 0; i < s.n_textures; ++i) a.blocked &= t->block_texels[i] != nullptr;
  a.ref = t->ref_blocks;
  a.inv_t = 1.0f / temperature;
  a.t2 = (float)(1.4426950408889634 / (double)temperature);
  a.w_e = lw ? lw[0] : 1.0f;
  a.w_c = lw ? lw[1] : 1.0f;
  a.w_cde = lw ? lw[2] : 1.0f;
  a.w_cdc = lw ? lw[3] : 1.0f;
  a.inv_ne = (float)(1.0 / ((double)n * s.endpoint_dim));
  a.inv_nc = (float)(1.0 / ((double)n * 16.0 * s.channels));
  a.losses = losses;
  int nf[2] = {0, 0};
  for (int i = 0; i < s.n_textures; ++i) {
    const int k = s.formats[i] == NTBC_BC1 ? 0 : 1;
    a.tex_of[k][nf[k]++] = i;
  }
  a.n_bc1 = nf[0];
  const dim3 grid((unsigned)loss_blocks(n, nf[0] + nf[1]));
  if (nf[0] > 0 && nf[1] > 0) hipLaunchKernelGGL(k_loss_grad_mixed, grid, dim3(64 * (nf[0] + nf[1])), 0, strm, a);
  else if (nf[0] > 0) hipLaunchKernelGGL(k_loss_grad<3>, grid, dim3(64 * nf[0]), 0, strm, a);
  else hipLaunchKernelGGL(k_loss_grad<1>, grid, dim3(64 * nf[1]), 0, strm, a);
  return check_launch("k_loss_grad");
}

// Naive-approach loss (stage 1 or 2) of heads [n][ld]; dsigmoid as loss_grad.
int naive_loss_grad(const Shape& s, const ntbc_targets* t, const float* heads, const int32_t* ids, int64_t n, int stage,
                    float* losses, float* dheads, hipStream_t strm, bool dsigmoid = false, int ld = 0,
                    bool losses_zeroed = false) {
  const int st = losses_zeroed ? NTBC_OK : fill(losses, 5, 0.0f, strm);
  if (st != NTBC_OK) return st;
  NaiveLossArgs a{};
  a.y = heads;
  a.dy = dheads;
  a.ids = ids;
  a.n = n;
  a.n_positions = s.n_positions;
  a.ld = ld > 0 ? ld : s.head_dim;
  a.E = s.endpoint_dim;
  a.T = s.n_textures;
  a.blocks_w = s.blocks_w;
  for (int i = 0; i < s.n_textures; ++i) {
    a.formats[i] = s.formats[i];
    a.ep_off[i] = s.ep_off[i];
    a.tex[i] = t->texels[i];
    a.btex[i] = t->block_texels[i];
  }
  a.blocked = 1;
  for (int i = 0; i < s.n_textures; ++i) a.blocked &= t->block_texels[i] != nullptr;
  a.inv_n = (float)(1.0 / ((double)n * 16.0 * s.channels));
  a.losses = losses;
  a.dsigmoid = dsigmoid ? 1 : 0;
  a.stage = stage;
  hipLaunchKernelGGL(k_loss_naive, dim3((unsigned)loss_blocks(n, s.n_textures)),
                     dim3(64 * s.n_textures), 0, strm, a);
  return check_launch("k_loss_naive");
}

int check_targets(const Shape& s, const ntbc_targets* t) {
  NTBC_REQUIRE(t != nullptr && t->ref_blocks != nullptr, "targets or ref_blocks is NULL");
  for (int i = 0; i < s.n_textures; ++i) NTBC_REQUIRE(t->texels[i] != nullptr, "targets texels[%d] is NULL", i);
  return NTBC_OK;
}

// ------------------------------------------------------------------------------------------ fused host
// Shapes the fused kernels take: hidden width 64 with two hidden layers, or 128 / 256 with three;
// in_dim <= 64 (four K-steps of features); head_dim <= 192.
constexpr int kFKS0 = 4, kFHT = kFHeadTiles;

struct FusedPlan {
  int hid, nh, L, S, T;
  PackTrainArgs pk;
  int64_t pack_n;             // u32x4
  int n_bias;
  FChunks fct, bct;
  int out_pad[kFMaxLayers];   // rows of dZ_k (position-contiguous)
  int64_t zrow[kFMaxLayers];
  int64_t z_rows;
};

bool fused_plan(const Shape& s, FusedPlan* fp) {
  const bool shape_ok = s.in_dim <= 16 * kFKS0 && s.head_dim <= 32 * kFHT &&
                        ((s.hidden == 64 && s.n_hidden == 2) || (s.hidden == 128 && s.n_hidden == 3) ||
                         (s.hidden == 256 && s.n_hidden == 3));
  if (!shape_ok) return false;
  FusedPlan& f = *fp;
  f = FusedPlan{};
  f.hid = s.hidden;
  f.nh = s.n_hidden - 1;
  f.L = s.n_layers;
  f.S = s.hidden / 16;
  f.T = s.hidden / 32;
  PackTrainArgs& a = f.pk;
  a.n_layers = f.L;
  int64_t off = 0;
  int boff = 0;
  for (int k = 0; k < f.L; ++k) {
    const bool head = k == f.L - 1;
    a.in_dim[k] = s.layer_in[k];
    a.out_dim[k] = s.layer_out[k];
    a.w_off[k] = s.w_off[k];
    a.b_off[k] = s.b_off[k];
    a.f_otiles[k] = head ? kFHT : f.T;
    a.f_ksteps[k] = k == 0 ? kFKS0 : f.S;
    a.f_off[k] = off;
    off += (int64_t)a.f_otiles[k] * a.f_ksteps[k] * 64;
    a.bias_off[k] = boff;
    boff += a.f_otiles[k] * 32;
    f.out_pad[k] = head ? 32 * kFHT : f.hid;
  }
  for (int k = 0; k < f.L; ++k) {
    a.b_otiles[k] = k == 0 ? (kFKS0 + 1) / 2 : f.T;
    a.b_ksteps[k] = f.out_pad[k] / 16;
    a.b_off2[k] = off;
    off += (int64_t)a.b_otiles[k] * a.b_ksteps[k] * 64;
  }
  f.pack_n = off;
  f.n_bias = boff;
  int64_t zr = 0;
  for (int k = 0; k < f.L; ++k) {
    f.zrow[k] = zr;
    zr += f.out_pad[k];
  }
  f.z_rows = zr;
  auto add = [](FChunks& ct, int64_t src, int ot, int ks) {
    for (int t = 0; t < ot; t += kFChunkTiles) {
      ct.src[ct.n] = src + (int64_t)t * ks * 64;
      ct.len[ct.n] = std::min(kFChunkTiles, ot - t) * ks * 64;
      ct.cap = std::max(ct.cap, ct.len[ct.n]);
      ++ct.n;
    }
  };
  for (int k = 0; k < f.L; ++k) add(f.fct, a.f_off[k], a.f_otiles[k], a.f_ksteps[k]);
  for (int k = f.L - 1; k >= 0; --k) add(f.bct, a.b_off2[k], a.b_otiles[k], a.b_ksteps[k]);
  f.fct.cap = f.bct.cap = std::max(f.fct.cap, f.bct.cap);
  return f.fct.n <= kFMaxChunks && f.bct.n <= kFMaxChunks;
}

// Workspace of the fused path for `batch` positions (bytes), laid out by fused_layout.
struct FusedLayout {
  int64_t pack, bias, y, dz, xt, ht, dzt, masks, dx, part, dbpart, total;  // byte offsets
  int64_t bpad;
  int splits, k_split, n_tiles;
};

FusedLayout fused_layout(const Shape& s, const FusedPlan& f, int64_t batch) {
  FusedLayout l{};
  l.bpad = ceil_div(std::max<int64_t>(batch, 1), kFPos) * kFPos;
  int64_t o = 1024;  // after the QAT statistics at the start of the workspace
  auto take = [&](int64_t bytes) {
    const int64_t r = o;
    o += (bytes + 255) / 256 * 256;
    return r;
  };
  l.pack = take(f.pack_n * 16);
  l.bias = take((int64_t)f.n_bias * 4);
  l.y = take(l.bpad * kFHeadLd * 4);
  l.dz = take(l.bpad * kFHeadLd * 4);
  l.xt = take((int64_t)16 * kFKS0 * l.bpad * 2);
  l.ht = take((int64_t)(f.L - 1) * f.hid * l.bpad * 2);
  l.dzt = take(f.z_rows * l.bpad * 2);
  l.masks = take((l.bpad / 32) * (f.L - 1) * (f.T / 2) * 64 * 4);
  l.dx = take(l.bpad * s.in_dim * 4);
  l.n_tiles = 0;
  for (int k = 0; k < f.L; ++k) l.n_tiles += (int)(ceil_div(s.layer_out[k], 128) * ceil_div(s.layer_in[k], 128));
  int splits = (int)std::max<int64_t>(1, std::min<int64_t>(512 / l.n_tiles, l.bpad / 256));
  l.k_split = (int)(ceil_div(ceil_div(l.bpad, splits), kDwK) * kDwK);
  l.splits = (int)ceil_div(l.bpad, l.k_split);
  l.part = take((int64_t)l.n_tiles * l.splits * 128 * 128 * 4);
  l.dbpart = take((int64_t)l.n_tiles * l.splits * 128 * 4);
  l.total = o;
  return l;
}

typedef void (*FwdKernel)(FwdArgs);
typedef void (*BwdKernel)(BwdArgs);

void fused_kernels(int hid, FwdKernel* fk, BwdKernel* bk) {
  if (hid == 64) {
    *fk = k_train_fwd<64, kFKS0, 1, kFHT>;
    *bk = k_train_bwd<64, kFKS0, 1, kFHT>;
  } else if (hid == 128) {
    *fk = k_train_fwd<128, kFKS0, 2, kFHT>;
    *bk = k_train_bwd<128, kFKS0, 2, kFHT>;
  } else {
    *fk = k_train_fwd<256, kFKS0, 2, kFHT>;
    *bk = k_train_bwd<256, kFKS0, 2, kFHT>;
  }
}

// Forward of the batch: packs the weights, then heads into y ([n][y_ld]); activations, masks and the
// layer-0 inputs stay in the workspace for fused_backward.  zero_losses: five floats the pack kernel
// zeroes on the way (a training step's loss sums, so the loss needs no fill of its own).
int fused_forward(Ctx& c, const FusedPlan& f, const float* grid, const float* weights, bool qat, const int32_t* ids,
                  float* y, int y_ld, float* zero_losses = nullptr) {
  const Shape& s = c.s;
  const FusedLayout l = fused_layout(s, f, c.n);
  char* ws = reinterpret_cast<char*>(c.ws);
  int st;
  if (qat) {
    st = qat_range(s, grid, c.stats(), c.strm);
    if (st != NTBC_OK) return st;
  }
  PackTrainArgs pk = f.pk;
  pk.w = weights;
  pk.pack = reinterpret_cast<u32x4*>(ws + l.pack);
  pk.bias = reinterpret_cast<float*>(ws + l.bias);
  pk.zero5 = zero_losses;
  hipLaunchKernelGGL(k_pack_train, dim3(64, 2 * f.L), dim3(256), 0, c.strm, pk);
  st = check_launch("k_pack_train");
  if (st != NTBC_OK) return st;
  FwdArgs a{};
  a.grid = grid;
  a.stats = qat ? c.stats() : nullptr;
  a.ids = ids;
  a.n = c.n;
  a.n_positions = s.n_positions;
  a.n_levels = s.n_levels;
  a.base_res = s.base_res;
  a.F = s.n_features;
  a.blocks_w = s.blocks_w;
  a.blocks_h = s.blocks_h;
  a.shift_x = pow2_shift(s, s.blocks_w);
  a.shift_y = pow2_shift(s, s.blocks_h);
  a.in_dim = s.in_dim;
  for (int i = 0; i <= s.n_levels; ++i) a.level_offset[i] = s.level_offset[i];
  a.wpack = pk.pack;
  a.bias = pk.bias;
  for (int k = 0; k < f.L; ++k) a.bias_off[k] = f.pk.bias_off[k];
  a.n_layers = f.L;
  a.head_dim = s.head_dim;
  a.n_bias = f.n_bias;
  a.bpad = l.bpad;
  a.xt = reinterpret_cast<uint16_t*>(ws + l.xt);
  a.ht = reinterpret_cast<uint16_t*>(ws + l.ht);
  a.masks = reinterpret_cast<uint32_t*>(ws + l.masks);
  a.y = y;
  a.y_ld = y_ld;
  a.ct = f.fct;
  FwdKernel fk;
  BwdKernel bk;
  fused_kernels(f.hid, &fk, &bk);
  const size_t lds = (size_t)2 * f.fct.cap * 16 + (size_t)kFW * kPatchBytes + (size_t)f.n_bias * 4;
  NTBC_HIP(hipFuncSetAttribute((const void*)fk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(fk, dim3((unsigned)(l.bpad / kFPos)), dim3(64 * kFW), lds, c.strm, a);
  return check_launch("k_train_fwd");
}

// A second stream of the current device (default priority) with a fork and a join event, created on
// first use and kept until the process ends: the grid scatter runs on it beside the weight-gradient
// products.  `lock` is held from the fork to the join, so that calls from several host threads do not
// interleave their uses of the two events.
struct SideStream {
  hipStream_t s;
  hipEvent_t fork, join;
  std::mutex lock;
};

int side_stream(SideStream** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static SideStream table[kMaxDevices];
  static bool made[kMaxDevices];
  int dev = 0;
  NTBC_HIP(hipGetDevice(&dev));
  NTBC_REQUIRE(dev >= 0 && dev < kMaxDevices, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> g(mu);
  if (!made[dev]) {
    NTBC_HIP(hipStreamCreateWithFlags(&table[dev].s, hipStreamNonBlocking));
    NTBC_HIP(hipEventCreateWithFlags(&table[dev].fork, hipEventDisableTiming));
    NTBC_HIP(hipEventCreateWithFlags(&table[dev].join, hipEventDisableTiming));
    made[dev] = true;
  }
  *out = &table[dev];
  return NTBC_OK;
}

// Backward of the batch from dZ of the head ([n][dz_ld]); the forward's workspace contents must be
// current.  ADDS the gradients to d_grid and to d_weights, or writes d_weights (assign_dw; then dw_flag,
// when set, becomes 1 if a weight gradient is not finite).  The fine levels' grid scatter (FP32 atomics from
// dX) and the weight products (from the stored activations and dZ) are independent: in atomic mode the
// scatter runs on the side stream, forked after the coarse levels' pass and joined back before
// returning.
int fused_backward(Ctx& c, const FusedPlan& f, const float* grid, bool qat, const int32_t* ids, const float* dz,
                   int dz_ld, float* d_grid, float* d_weights, bool assign_dw = false, float* dw_flag = nullptr) {
  const Shape& s = c.s;
  const FusedLayout l = fused_layout(s, f, c.n);
  char* ws = reinterpret_cast<char*>(c.ws);
  BwdArgs b{};
  b.dz = dz;
  b.dz_ld = dz_ld;
  b.head_dim = s.head_dim;
  b.n = c.n;
  b.bpad = l.bpad;
  b.wpack = reinterpret_cast<const u32x4*>(ws + l.pack);
  b.masks = reinterpret_cast<const uint32_t*>(ws + l.masks);
  b.dzt = reinterpret_cast<uint16_t*>(ws + l.dzt);
  for (int k = 0; k < f.L; ++k) b.zrow[k] = f.zrow[k];
  b.dx = reinterpret_cast<float*>(ws + l.dx);
  b.in_dim = s.in_dim;
  b.n_layers = f.L;
  b.ct = f.bct;
  FwdKernel fk;
  BwdKernel bk;
  fused_kernels(f.hid, &fk, &bk);
  const size_t lds = (size_t)2 * f.bct.cap * 16 + (size_t)kFW * kPatchBytes;
  NTBC_HIP(hipFuncSetAttribute((const void*)bk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(bk, dim3((unsigned)(l.bpad / kFPos)), dim3(64 * kFW), lds, c.strm, b);
  int st = check_launch("k_train_bwd");
  if (st != NTBC_OK) return st;
  SideStream* side = nullptr;
  if (!c.det) {
    st = side_stream(&side);
    if (st != NTBC_OK) return st;
  }
  std::unique_lock<std::mutex> hold;
  if (side) {
    hold = std::unique_lock<std::mutex>(side->lock);
    st = scatter_grid(c, grid, qat, ids, b.dx, d_grid, 1);
    NTBC_HIP(hipEventRecord(side->fork, c.strm));
    NTBC_HIP(hipStreamWaitEvent(side->s, side->fork, 0));
    Ctx cs = c;
    cs.strm = side->s;
    if (st == NTBC_OK) st = scatter_grid(cs, grid, qat, ids, b.dx, d_grid, 2);
    NTBC_HIP(hipEventRecord(side->join, side->s));
    if (st != NTBC_OK) {
      NTBC_HIP(hipStreamWaitEvent(c.strm, side->join, 0));
      return st;
    }
  } else {
    st = scatter_grid(c, grid, qat, ids, b.dx, d_grid);
    if (st != NTBC_OK) return st;
  }
  DwArgs d{};
  const uint16_t* xt = reinterpret_cast<const uint16_t*>(ws + l.xt);
  const uint16_t* ht = reinterpret_cast<const uint16_t*>(ws + l.ht);
  int tile0 = 0;
  for (int k = 0; k < f.L; ++k) {
    DwJob& J = d.job[k];
    J.a = b.dzt + f.zrow[k] * l.bpad;
    J.a_rows = f.out_pad[k];
    J.b = k == 0 ? xt : ht + (int64_t)(k - 1) * f.hid * l.bpad;
    J.b_rows = k == 0 ? 16 * kFKS0 : f.hid;
    J.M = s.layer_out[k];
    J.N = s.layer_in[k];
    J.tiles_n = (int)ceil_div(J.N, 128);
    J.tile0 = tile0;
    tile0 += (int)ceil_div(J.M, 128) * J.tiles_n;
    J.c = d_weights + s.w_off[k];
    J.db = d_weights + s.b_off[k];
  }
  d.n_jobs = f.L;
  d.n_tiles = tile0;
  d.splits = l.splits;
  d.k_split = l.k_split;
  d.bpad = l.bpad;
  d.K = l.bpad;
  d.part = reinterpret_cast<float*>(ws + l.part);
  d.dbpart = reinterpret_cast<float*>(ws + l.dbpart);
  d.assign = assign_dw ? 1 : 0;
  d.flag = dw_flag;
  hipLaunchKernelGGL(k_train_dw, dim3((unsigned)(d.n_tiles * d.splits)), dim3(256), 0, c.strm, d);
  st = check_launch("k_train_dw");
  if (st == NTBC_OK) {
    hipLaunchKernelGGL(k_train_dw_reduce, dim3(64, (unsigned)d.n_tiles), dim3(256), 0, c.strm, d);
    st = check_launch("k_train_dw_reduce");
  }
  // the caller's stream waits for the scatter
  if (side) NTBC_HIP(hipStreamWaitEvent(c.strm, side->join, 0));
  return st;
}

// dZ = dY * Y (1 - Y) with row strides (ntbc_backward: d_heads [n][head_dim], heads [n][y_ld]).
__global__ void k_dsigmoid_ld(const float* __restrict__ dy, int ld_dy, const float* __restrict__ y, int ld_y,
                              float* __restrict__ dz, int ld_dz, int64_t n, int cols) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n * cols; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols;
    const int k = (int)(i % cols);
    const float yv = y[r * ld_y + k];
    dz[r * ld_dz + k] = dy[r * ld_dy + k] * yv * (1.0f - yv);
  }
}


// Byte offset of the deterministic scatter's region (after the unfused and fused layouts).
int64_t det_offset(const Shape& s, int64_t batch) {
  int64_t bytes = train_layout(s, batch).total * (int64_t)sizeof(float);
  FusedPlan f;
  if (fused_plan(s, &f)) bytes = std::max(bytes, fused_layout(s, f, batch).total);
  return (bytes + 255) / 256 * 256;
}

// Byte offset of the coarse scatter's per-block sums (after the deterministic scatter's region); one row
// of at most kCoarseLds bytes per block.
int64_t coarse_offset(const Shape& s, int64_t batch) {
  return det_offset(s, batch) + 256 + (s.grid_vertices * s.n_features * 8 + 255) / 256 * 256;
}

}  // namespace

namespace ntbc {
// The unfused and fused layouts share the workspace; the deterministic scatter's 64-bit sums and the
// coarse scatter's per-block sums follow.
int64_t train_workspace_bytes(const Shape& s, int64_t batch) {
  return coarse_offset(s, batch) + (int64_t)kCoarseBlocks * kCoarseLds;
}
}  // namespace ntbc

extern "C" int ntbc_forward(const ntbc_model_desc* d, const float* grid, const float* weights, int32_t qat,
                            int32_t precision, const int32_t* ids, int32_t n, float* heads_out, void* workspace,
                            size_t workspace_bytes, void* stream) {
  Ctx c;
  int st = check_common(d, precision, ids, n, workspace, workspace_bytes, &c);
  if (st != NTBC_OK) return st;
  NTBC_REQUIRE(grid && weights, "grid or weights is NULL");
  if (n == 0) return NTBC_OK;
  NTBC_REQUIRE(heads_out != nullptr, "heads_out is NULL");
  c.strm = as_stream(stream);
  FusedPlan f;
  if (c.bf16 && fused_plan(c.s, &f)) return fused_forward(c, f, grid, weights, qat != 0, ids, heads_out, c.s.head_dim);
  return forward(c, grid, weights, qat != 0, ids, heads_out);
}

extern "C" int ntbc_backward(const ntbc_model_desc* d, const float* grid, const float* weights, int32_t qat,
                             int32_t precision, const int32_t* ids, int32_t n, const float* d_heads, float* d_grid,
                             float* d_weights, void* workspace, size_t workspace_bytes, void* stream) {
  Ctx c;
  int st = check_common(d, precision, ids, n, workspace, workspace_bytes, &c);
  if (st != NTBC_OK) return st;
  NTBC_REQUIRE(grid && weights && d_grid && d_weights, "grid, weights, d_grid or d_weights is NULL");
  if (n == 0) return NTBC_OK;
  NTBC_REQUIRE(d_heads != nullptr, "d_heads is NULL");
  c.strm = as_stream(stream);
  FusedPlan f;
  if (c.bf16 && fused_plan(c.s, &f)) {
    const FusedLayout l = fused_layout(c.s, f, c.n);
    char* ws = reinterpret_cast<char*>(c.ws);
    float* y = reinterpret_cast<float*>(ws + l.y);
    float* dz = reinterpret_cast<float*>(ws + l.dz);
    st = fused_forward(c, f, grid, weights, qat != 0, ids, y, kFHeadLd);
    if (st != NTBC_OK) return st;
    hipLaunchKernelGGL(k_dsigmoid_ld, dim3((unsigned)std::min<int64_t>(ceil_div(c.n * c.s.head_dim, 256), 4096)), dim3(256), 0,
                       c.strm, d_heads, c.s.head_dim, y, kFHeadLd, dz, kFHeadLd, c.n, c.s.head_dim);
    st = check_launch("k_dsigmoid_ld");
    if (st != NTBC_OK) return st;
    return fused_backward(c, f, grid, qat != 0, ids, dz, kFHeadLd, d_grid, d_weights);
  }
  float* y = c.ws + c.lay.y;
  st = forward(c, grid, weights, qat != 0, ids, y);
  if (st != NTBC_OK) return st;
  const int64_t ny = c.n * c.s.head_dim;
  hipLaunchKernelGGL(k_dsigmoid, dim3((unsigned)std::min<int64_t>(ceil_div(ny, 256), 4096)), dim3(256), 0, c.strm, d_heads, y,
                     c.ws + c.lay.dy, ny);
  st = check_launch("k_dsigmoid");
  if (st != NTBC_OK) return st;
  return backward(c, grid, weights, qat != 0, ids, d_grid, d_weights);
}

extern "C" int ntbc_loss_grad(const ntbc_model_desc* d, const ntbc_targets* t, const float* heads, const int32_t* ids,
                              int32_t n, float temperature, const float* loss_weights, float* losses_out,
                              float* d_heads_out, void* stream) {
  Shape s;
  int st = make_shape(d, &s);
  if (st != NTBC_OK) return st;
  st = check_targets(s, t);
  if (st != NTBC_OK) return st;
  NTBC_REQUIRE(n >= 0, "n %d < 0", n);
  NTBC_REQUIRE(temperature > 0.0f, "temperature must be positive");
  NTBC_REQUIRE(losses_out != nullptr, "losses_out is NULL");
  if (n == 0) return fill(losses_out, 5, 0.0f, as_stream(stream));
  NTBC_REQUIRE(heads && ids && d_heads_out, "heads, ids or d_heads_out is NULL");
  return loss_grad(s, t, heads, ids, n, temperature, loss_weights, losses_out, d_heads_out, as_stream(stream));
}

extern "C" int ntbc_naive_loss_grad(const ntbc_model_desc* d, const ntbc_targets* t, const float* heads,
                                    const int32_t* ids, int32_t n, int32_t stage, float* losses_out, float* d_heads_out,
                                    void* stream) {
  Shape s;
  int st = make_shape(d, &s);
  if (st != NTBC_OK) return st;
  NTBC_REQUIRE(s.naive, "ntbc_naive_loss_grad needs variant NTBC_NAIVE");
  NTBC_REQUIRE(stage == 1 || stage == 2, "stage %d is not 1 or 2", stage);
  st = check_targets(s, t);
  if (st != NTBC_OK) return st;
  NTBC_REQUIRE(n >= 0, "n %d < 0", n);
  NTBC_REQUIRE(losses_out != nullptr, "losses_out is NULL");
  if (n == 0) return fill(losses_out, 5, 0.0f, as_stream(stream));
  NTBC_REQUIRE(heads && ids && d_heads_out, "heads, ids or d_heads_out is NULL");
  return naive_loss_grad(s, t, heads, ids, n, stage, losses_out, d_heads_out, as_stream(stream));
}

extern "C" int ntbc_train_step(const ntbc_model_desc* d, const ntbc_train_state* tsd, const ntbc_targets* t,
                               const int32_t* batch_ids, int32_t batch, int64_t step, const ntbc_hparams* h,
                               float* losses_out, void* workspace, size_t workspace_bytes, void* stream) {
  NTBC_REQUIRE(h != nullptr && tsd != nullptr, "hparams or state is NULL");
  Ctx c;
  int st = check_common(d, h->precision, batch_ids, batch, workspace, workspace_bytes, &c);
  if (st != NTBC_OK) return st;
  st = check_targets(c.s, t);
  if (st != NTBC_OK) return st;
  NTBC_REQUIRE(batch > 0, "batch must be positive");
  NTBC_REQUIRE(step >= 0, "step must be >= 0");
  NTBC_REQUIRE(tsd->grid && tsd->weights && tsd->m_grid && tsd->v_grid && tsd->m_weights && tsd->v_weights &&
                   tsd->d_grid && tsd->d_weights,
               "a train-state pointer is NULL");
  NTBC_REQUIRE(losses_out != nullptr, "losses_out is NULL");
  NTBC_REQUIRE(h->temperature > 0.0f && h->total_steps > 0 && h->warmup >= 0, "bad temperature or schedule");
  c.strm = as_stream(stream);
  c.det = h->deterministic != 0;
  const Shape& s = c.s;
  const bool qat = h->qat != 0;
  const int64_t ng = s.grid_vertices * s.n_features;
  // naive approach: stage 2 (quantised weights, endpoint head only) from step stage2_from on
  const int stage = s.naive && step >= h->stage2_from ? 2 : 1;
  FusedPlan f;
  if (c.bf16 && fused_plan(s, &f)) {
    // bfloat16 products with the layers chained in registers
    const FusedLayout l = fused_layout(s, f, c.n);
    char* ws = reinterpret_cast<char*>(c.ws);
    float* y = reinterpret_cast<float*>(ws + l.y);
    float* dz = reinterpret_cast<float*>(ws + l.dz);
    // the pack kernel zeroes the loss sums; the weight products write d_weights (no fill) and flag a
    // non-finite weight gradient (no separate check)
    st = fused_forward(c, f, tsd->grid, tsd->weights, qat, batch_ids, y, kFHeadLd, losses_out);
    if (st != NTBC_OK) return st;
    st = s.naive ? naive_loss_grad(s, t, y, batch_ids, c.n, stage, losses_out, dz, c.strm, true, kFHeadLd, true)
                 : loss_grad(s, t, y, batch_ids, c.n, h->temperature, h->loss_weights, losses_out, dz, c.strm, true,
                             kFHeadLd, true);
    if (st != NTBC_OK) return st;
    st = fill(tsd->d_grid, ng, 0.0f, c.strm);
    if (st != NTBC_OK) return st;
    st = fused_backward(c, f, tsd->grid, qat, batch_ids, dz, kFHeadLd, tsd->d_grid, tsd->d_weights, true,
                        losses_out + 4);
    if (st != NTBC_OK) return st;
  } else {
    float* y = c.ws + c.lay.y;
    st = forward(c, tsd->grid, tsd->weights, qat, batch_ids, y);
    if (st != NTBC_OK) return st;
    // dL/dZ of the head pre-activations straight from the loss kernel (the sigmoid derivative fused)
    st = s.naive ? naive_loss_grad(s, t, y, batch_ids, c.n, stage, losses_out, c.ws + c.lay.dy, c.strm, true)
                 : loss_grad(s, t, y, batch_ids, c.n, h->temperature, h->loss_weights, losses_out, c.ws + c.lay.dy,
                             c.strm, true);
    if (st != NTBC_OK) return st;
    st = fill(tsd->d_grid, ng, 0.0f, c.strm);
    if (st == NTBC_OK) st = fill(tsd->d_weights, s.n_weights, 0.0f, c.strm);
    if (st != NTBC_OK) return st;
    st = backward(c, tsd->grid, tsd->weights, qat, batch_ids, tsd->d_grid, tsd->d_weights);
    if (st != NTBC_OK) return st;
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)std::min<int64_t>(ceil_div(s.n_weights, 256), 1024)), dim3(256),
                       0, c.strm, tsd->d_weights, s.n_weights, losses_out + 4);
  }
  // learning rates of this step: linear warm-up, then cosine annealing to 0
  auto lr_at = [&](double lr0) {
    if (step < h->warmup) return lr0 * (double)(step + 1) / h->warmup;
    const double span = h->total_steps - h->warmup > 0 ? (double)(h->total_steps - h->warmup) : 1.0;
    return lr0 * 0.5 * (1.0 + std::cos(M_PI * (double)(step - h->warmup) / span));
  };
  const double tt = (double)step + 1.0;
  AdamArgs aa{};
  aa.b1 = h->beta1;
  aa.b2 = h->beta2;
  aa.eps = h->eps;
  aa.bc1 = (float)(1.0 / (1.0 - std::pow((double)h->beta1, tt)));
  aa.bc2 = (float)(1.0 / (1.0 - std::pow((double)h->beta2, tt)));
  aa.flag = losses_out + 4;
  const float lr_w = (float)lr_at(h->lr_mlp);
  if (stage == 2) {
    // only the endpoint head's rows of the last layer: W rows 0..E-1 and b[0..E-1], each contiguous
    const int last = s.n_layers - 1;
    const int64_t nw = (int64_t)s.endpoint_dim * s.layer_in[last];
    auto part = [&](int64_t off, int64_t n) {
      return AdamPart{tsd->weights + off, tsd->d_weights + off, tsd->m_weights + off, tsd->v_weights + off, n, lr_w, 0};
    };
    return adam(part(s.w_off[last], nw), part(s.b_off[last], s.endpoint_dim), aa, c.strm);
  }
  // the weights and the grid in one launch, each with its learning rate
  const AdamPart pw{tsd->weights, tsd->d_weights, tsd->m_weights, tsd->v_weights, s.n_weights, lr_w, 0};
  const AdamPart pg{tsd->grid, tsd->d_grid, tsd->m_grid, tsd->v_grid, ng, (float)lr_at(h->lr_grid), 0};
  return adam(pw, pg, aa, c.strm);
}

// ------------------------------------------------------------------------------------------ paper layout
// Training of one model of the paper's own layout (Sec. 3.2, Sec. 3.4, Sec. 4.1): the endpoint network
// runs as a model over the block grid and the colour network as a model over the texel grid (4 blocks_w
// x 4 blocks_h cells), both through the FP32 forward / backward above with SELU hidden layers; the heads
// of the batch's blocks are assembled in the NTBC layout for the loss, and its gradient is split back.
namespace {

void set_outputs(Shape* s, int out) {
  s->head_dim = out;
  s->layer_out[s->n_layers - 1] = out;
  int64_t w = 0;
  for (int k = 0; k < s->n_layers; ++k) {
    s->w_off[k] = w;
    w += (int64_t)s->layer_in[k] * s->layer_out[k];
    s->b_off[k] = w;
    w += s->layer_out[k];
  }
  s->n_weights = w;
}

// ep: the endpoint network (its grid over the block grid, E outputs); col: the colour network (its grid
// over the texel grid, C outputs); loss: the NTBC head layout of the model's textures (E + 16 C).
int faithful_shapes(const ntbc_faithful_desc* d, Shape* ep, Shape* col, Shape* loss) {
  NTBC_REQUIRE(d != nullptr, "desc is NULL");
  NTBC_REQUIRE(d->grid_dtype == NTBC_GRID_F32, "the paper layout trains FP32 master grids (grid_dtype %d)",
               d->grid_dtype);
  NTBC_REQUIRE(d->blocks_w >= 1 && d->blocks_h >= 1 && 16 * (int64_t)d->blocks_w * d->blocks_h < (1ll << 31),
               "block grid %dx%d: its texels must number below 2^31", d->blocks_w, d->blocks_h);
  NTBC_REQUIRE(d->n_textures >= 1 && d->n_textures <= NTBC_MAX_TEXTURES, "n_textures %d out of 1..%d", d->n_textures,
               NTBC_MAX_TEXTURES);
  ntbc_model_desc m{};
  m.n_levels = d->ep_levels;
  m.base_res = d->ep_base_res;
  m.n_features = 2;
  m.grid_dtype = NTBC_GRID_F32;
  m.hidden_width = 64;
  m.n_hidden = 3;
  m.n_textures = d->n_textures;
  for (int t = 0; t < d->n_textures; ++t) m.formats[t] = d->formats[t];
  m.blocks_w = d->blocks_w;
  m.blocks_h = d->blocks_h;
  m.variant = NTBC_NTBC;
  int st = make_shape(&m, loss);
  if (st != NTBC_OK) return st;
  *ep = *loss;
  set_outputs(ep, loss->endpoint_dim);
  m.n_levels = d->col_levels;
  m.base_res = d->col_base_res;
  m.blocks_w = 4 * d->blocks_w;
  m.blocks_h = 4 * d->blocks_h;
  st = make_shape(&m, col);
  if (st != NTBC_OK) return st;
  set_outputs(col, loss->channels);
  return NTBC_OK;
}

struct FaithfulTrainLayout {
  int64_t ep, col, tids, heads, dheads, total;  // byte offsets
};

FaithfulTrainLayout faithful_train_layout(const Shape& ep, const Shape& col, const Shape& loss, int64_t batch) {
  FaithfulTrainLayout l{};
  int64_t o = 0;
  auto take = [&](int64_t bytes) {
    const int64_t r = o;
    o += (bytes + 255) / 256 * 256;
    return r;
  };
  l.ep = take(train_workspace_bytes(ep, batch));
  l.col = take(train_workspace_bytes(col, 16 * batch));
  l.tids = take(16 * batch * 4);
  l.heads = take(batch * loss.head_dim * 4);
  l.dheads = take(batch * loss.head_dim * 4);
  l.total = o;
  return l;
}

Ctx faithful_ctx(const Shape& s, int64_t n, char* ws, hipStream_t strm, bool det) {
  Ctx c;
  c.s = s;
  c.lay = train_layout(s, n);
  c.ws = reinterpret_cast<float*>(ws);
  c.n = n;
  c.strm = strm;
  c.bf16 = false;
  c.det = det;
  c.det_off = det_offset(s, n);
  c.selu = true;
  return c;
}

Ctx faithful_colour_ctx(const Shape& s, int64_t n, char* ws, hipStream_t strm, bool det) {
  Ctx c = faithful_ctx(s, n, ws, strm, det);
  c.texel_blocks = true;
  return c;
}

// The colour network's positions: texel i = 4y + x of block ids[p] is cell (4 bx + x, 4 by + y) of the
// texel grid.
__global__ void k_texel_ids(const int32_t* __restrict__ ids, int64_t n, int blocks_w, int64_t n_positions,
                            int32_t* __restrict__ tids) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < 16 * n; e += (int64_t)gridDim.x * blockDim.x) {
    const int id = clamp_id(ids[e >> 4], n_positions);
    const int i = (int)(e & 15), bx = id % blocks_w, by = id / blocks_w;
    tids[e] = (4 * by + (i >> 2)) * (4 * blocks_w) + 4 * bx + (i & 3);
  }
}

// Heads [n][E + 16 C] from the endpoint outputs [n][E] and the colour outputs [16 n][C] (those of block p,
// texel-major with C channels each, are its heads E .. E + 16 C - 1 in order); split = 1: the reverse.
__global__ void k_fa_heads(float* __restrict__ heads, float* __restrict__ ye, float* __restrict__ yc, int64_t n,
                           int E, int C, int split) {
  const int H = E + 16 * C;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * H; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / H;
    const int k = (int)(e - p * H);
    float* part = k < E ? ye + p * E + k : yc + p * 16 * C + (k - E);
    if (split) *part = heads[e];
    else heads[e] = *part;
  }
}

// Learning rate of `step` (0-based): linear warm-up, then cosine annealing to 0 at total_steps.
double schedule_lr(const ntbc_hparams* h, int64_t step, double lr0) {
  if (step < h->warmup) return lr0 * (double)(step + 1) / h->warmup;
  const double span = h->total_steps - h->warmup > 0 ? (double)(h->total_steps - h->warmup) : 1.0;
  return lr0 * 0.5 * (1.0 + std::cos(M_PI * (double)(step - h->warmup) / span));
}

}  // namespace

extern "C" int ntbc_faithful_train_size(const ntbc_faithful_desc* d, int32_t batch, size_t* workspace_bytes) {
  NTBC_REQUIRE(workspace_bytes != nullptr, "workspace_bytes is NULL");
  NTBC_REQUIRE(batch >= 1, "batch %d < 1", batch);
  Shape ep, col, loss;
  const int st = faithful_shapes(d, &ep, &col, &loss);
  if (st != NTBC_OK) return st;
  *workspace_bytes = (size_t)faithful_train_layout(ep, col, loss, batch).total;
  return NTBC_OK;
}

extern "C" int ntbc_faithful_train_step(const ntbc_faithful_desc* d, const ntbc_faithful_train_state* tsd,
                                        const ntbc_targets* t, const int32_t* batch_ids, int32_t batch, int64_t step,
                                        const ntbc_hparams* h, float* losses_out, void* workspace,
                                        size_t workspace_bytes, void* stream) {
  NTBC_REQUIRE(h != nullptr && tsd != nullptr, "hparams or state is NULL");
  Shape ep, col, loss;
  int st = faithful_shapes(d, &ep, &col, &loss);
  if (st != NTBC_OK) return st;
  if (h->precision != NTBC_FP32)
    return fail(NTBC_EUNSUPPORTED, "the paper layout trains with FP32 products (precision %d)", h->precision);
  st = check_targets(loss, t);
  if (st != NTBC_OK) return st;
  NTBC_REQUIRE(batch > 0 && batch_ids != nullptr, "batch must be positive, with ids");
  NTBC_REQUIRE(step >= 0, "step must be >= 0");
  NTBC_REQUIRE(tsd->ep_grid && tsd->col_grid && tsd->ep_weights && tsd->col_weights && tsd->m_ep_grid && tsd->v_ep_grid &&
                   tsd->m_col_grid && tsd->v_col_grid && tsd->m_ep_weights && tsd->v_ep_weights && tsd->m_col_weights &&
                   tsd->v_col_weights && tsd->d_ep_grid && tsd->d_col_grid && tsd->d_ep_weights && tsd->d_col_weights,
               "a train-state pointer is NULL");
  NTBC_REQUIRE(losses_out != nullptr, "losses_out is NULL");
  NTBC_REQUIRE(h->temperature > 0.0f && h->total_steps > 0 && h->warmup >= 0, "bad temperature or schedule");
  const FaithfulTrainLayout l = faithful_train_layout(ep, col, loss, batch);
  if (workspace == nullptr || workspace_bytes < (size_t)l.total)
    return fail(NTBC_ENOWORKSPACE, "workspace needs %lld bytes", (long long)l.total);
  char* ws = static_cast<char*>(workspace);
  const hipStream_t strm = as_stream(stream);
  const bool det = h->deterministic != 0, qat = h->qat != 0;
  Ctx ce = faithful_ctx(ep, batch, ws + l.ep, strm, det);
  Ctx cc = faithful_colour_ctx(col, 16 * (int64_t)batch, ws + l.col, strm, det);
  int32_t* tids = reinterpret_cast<int32_t*>(ws + l.tids);
  float* heads = reinterpret_cast<float*>(ws + l.heads);
  float* dheads = reinterpret_cast<float*>(ws + l.dheads);
  float* ye = ce.ws + ce.lay.y;
  float* yc = cc.ws + cc.lay.y;
  const int E = loss.endpoint_dim, C = loss.channels;
  const unsigned hb = (unsigned)std::min<int64_t>(ceil_div((int64_t)batch * loss.head_dim, 256), 4096);
  hipLaunchKernelGGL(k_texel_ids, dim3((unsigned)std::min<int64_t>(ceil_div(16 * (int64_t)batch, 256), 4096)), dim3(256),
                     0, strm, batch_ids, (int64_t)batch, loss.blocks_w, loss.n_positions, tids);
  st = check_launch("k_texel_ids");
  if (st == NTBC_OK) st = forward(ce, tsd->ep_grid, tsd->ep_weights, qat, batch_ids, ye);
  if (st == NTBC_OK) st = forward(cc, tsd->col_grid, tsd->col_weights, qat, tids, yc);
  if (st != NTBC_OK) return st;
  hipLaunchKernelGGL(k_fa_heads, dim3(hb), dim3(256), 0, strm, heads, ye, yc, (int64_t)batch, E, C, 0);
  // dL/dZ of the output pre-activations of both networks, in the head layout, then split
  st = loss_grad(loss, t, heads, batch_ids, batch, h->temperature, h->loss_weights, losses_out, dheads, strm, true);
  if (st != NTBC_OK) return st;
  hipLaunchKernelGGL(k_fa_heads, dim3(hb), dim3(256), 0, strm, dheads, ce.ws + ce.lay.dy, cc.ws + cc.lay.dy,
                     (int64_t)batch, E, C, 1);
  const int64_t nge = ep.grid_vertices * 2, ngc = col.grid_vertices * 2;
  st = fill(tsd->d_ep_grid, nge, 0.0f, strm);
  if (st == NTBC_OK) st = fill(tsd->d_col_grid, ngc, 0.0f, strm);
  if (st == NTBC_OK) st = fill(tsd->d_ep_weights, ep.n_weights, 0.0f, strm);
  if (st == NTBC_OK) st = fill(tsd->d_col_weights, col.n_weights, 0.0f, strm);
  if (st == NTBC_OK) st = backward(ce, tsd->ep_grid, tsd->ep_weights, qat, batch_ids, tsd->d_ep_grid, tsd->d_ep_weights);
  if (st == NTBC_OK) st = backward(cc, tsd->col_grid, tsd->col_weights, qat, tids, tsd->d_col_grid, tsd->d_col_weights);
  if (st != NTBC_OK) return st;
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)std::min<int64_t>(ceil_div(ep.n_weights, 256), 1024)), dim3(256), 0,
                     strm, tsd->d_ep_weights, ep.n_weights, losses_out + 4);
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)std::min<int64_t>(ceil_div(col.n_weights, 256), 1024)), dim3(256), 0,
                     strm, tsd->d_col_weights, col.n_weights, losses_out + 4);
  const double tt = (double)step + 1.0;
  AdamArgs aa{};
  aa.b1 = h->beta1;
  aa.b2 = h->beta2;
  aa.eps = h->eps;
  aa.bc1 = (float)(1.0 / (1.0 - std::pow((double)h->beta1, tt)));
  aa.bc2 = (float)(1.0 / (1.0 - std::pow((double)h->beta2, tt)));
  aa.flag = losses_out + 4;
  struct Set {
    float *p, *g, *m, *v;
    int64_t n;
    bool grid;
  } sets[4] = {{tsd->ep_grid, tsd->d_ep_grid, tsd->m_ep_grid, tsd->v_ep_grid, nge, true},
               {tsd->col_grid, tsd->d_col_grid, tsd->m_col_grid, tsd->v_col_grid, ngc, true},
               {tsd->ep_weights, tsd->d_ep_weights, tsd->m_ep_weights, tsd->v_ep_weights, ep.n_weights, false},
               {tsd->col_weights, tsd->d_col_weights, tsd->m_col_weights, tsd->v_col_weights, col.n_weights, false}};
  AdamPart parts[4];
  for (int k = 0; k < 4; ++k) {
    const Set& q = sets[k];
    parts[k] = AdamPart{q.p, q.g, q.m, q.v, q.n, (float)schedule_lr(h, step, q.grid ? h->lr_grid : h->lr_mlp), 0};
  }
  st = adam(parts[0], parts[1], aa, strm);
  if (st == NTBC_OK) st = adam(parts[2], parts[3], aa, strm);
  return st;
}

extern "C" int ntbc_train_status(const float* losses, void* stream) {
  NTBC_REQUIRE(losses != nullptr, "losses is NULL");
  float flag = 0.0f;
  NTBC_HIP(hipMemcpyAsync(&flag, losses + 4, sizeof(float), hipMemcpyDeviceToHost, as_stream(stream)));
  NTBC_HIP(hipStreamSynchronize(as_stream(stream)));
  if (flag != 0.0f)
    return fail(NTBC_ENONFINITE, "the training step saw a non-finite loss or gradient; parameters and moments unchanged");
  return NTBC_OK;
}

extern "C" int ntbc_quantize_grid(const ntbc_model_desc* d, const float* grid, uint8_t* codes, float* scale,
                                  int32_t* zero, void* workspace, size_t workspace_bytes, void* stream) {
  Shape s;
  int st = make_shape(d, &s);
  if (st != NTBC_OK) return st;
  NTBC_REQUIRE(grid && codes && scale && zero, "NULL pointer argument");
  if (workspace == nullptr || workspace_bytes < 4 * NTBC_MAX_LEVELS * sizeof(float))
    return fail(NTBC_ENOWORKSPACE, "workspace needs %d bytes", (int)(4 * NTBC_MAX_LEVELS * sizeof(float)));
  hipStream_t strm = as_stream(stream);
  int* stats = static_cast<int*>(workspace);
  st = qat_range(s, grid, stats, strm);
  if (st != NTBC_OK) return st;
  const LevelArgs la = level_args(s);
  int64_t mx = 0;
  for (int l = 0; l < s.n_levels; ++l) mx = la.count[l] > mx ? la.count[l] : mx;
  hipLaunchKernelGGL(k_quantize, dim3((unsigned)std::min<int64_t>(ceil_div(mx, 256), 4096), s.n_levels), dim3(256), 0, strm,
                     grid, la, stats, codes);
  hipLaunchKernelGGL(k_export_qparams, dim3(1), dim3(64), 0, strm, stats, s.n_levels, scale, zero);
  return check_launch("ntbc_quantize_grid");
}

extern "C" int ntbc_batch_ids(uint64_t seed, int64_t step, int32_t batch, int64_t n_positions, int32_t* ids_out,
                              void* stream) {
  NTBC_REQUIRE(ids_out != nullptr || batch == 0, "ids_out is NULL");
  NTBC_REQUIRE(batch >= 0 && n_positions > 0 && n_positions <= 0x7FFFFFFF, "bad batch or n_positions");
  if (batch == 0) return NTBC_OK;
  uint64_t h = 0;
  const uint64_t parts[3] = {seed, 0xBA7C4ull, (uint64_t)step};
  for (uint64_t p : parts) h = splitmix_out((h ^ p) + kGamma);
  hipLaunchKernelGGL(k_batch_ids, dim3((unsigned)ceil_div(batch, 256)), dim3(256), 0, as_stream(stream), h, batch,
                     (uint64_t)n_positions, ids_out);
  return check_launch("ntbc_batch_ids");
}
