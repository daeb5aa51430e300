// Internal helpers shared by the HIP sources of libntbc: status reporting, argument checks, model
// shape arithmetic.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>

#include "ntbc.h"

namespace ntbc {

// Sets the thread-local message returned by ntbc_last_error() and returns `status`.
int fail(int status, const char* fmt, ...);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Checks the last kernel launch on the host side.
int check_launch(const char* what);

#define NTBC_REQUIRE(cond, ...)                                   \
  do {                                                            \
    if (!(cond)) return ::ntbc::fail(NTBC_EINVAL, __VA_ARGS__);   \
  } while (0)

#define NTBC_HIP(call)                                                                        \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return ::ntbc::fail(NTBC_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));          \
  } while (0)

// Derived sizes of a model description.
struct Shape {
  int n_levels, base_res, n_features, in_dim, hidden, n_hidden, n_layers;
  int n_textures, formats[NTBC_MAX_TEXTURES];
  int ep_off[NTBC_MAX_TEXTURES], ch_off[NTBC_MAX_TEXTURES];
  int endpoint_dim, channels, head_dim;
  int naive;  // NTBC_NAIVE: the weight head (16 * n_textures values) replaces the colour head
  int blocks_w, blocks_h;
  int64_t n_positions, grid_vertices, n_weights;
  int64_t level_offset[NTBC_MAX_LEVELS + 1];
  int layer_in[8], layer_out[8];
  int64_t w_off[8], b_off[8];
};

// Validates `d` and fills `s`; returns NTBC_OK or NTBC_EINVAL (with the message set).
int make_shape(const ntbc_model_desc* d, Shape* s);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// log2(2 * blocks) when that is a power of two and every numerator of the grid-corner arithmetic
// ((2b + 1) res - blocks, and the clamp bound (res - 1) 2 blocks) fits in 31 bits at the finest level,
// else -1: the corner computation then takes shifts instead of divisions.
inline int pow2_shift(const Shape& s, int blocks) {
  const int64_t den = 2 * (int64_t)blocks;
  const int64_t top = (int64_t)s.base_res << (s.n_levels - 1);
  if ((den & (den - 1)) != 0 || (2 * (int64_t)blocks + 1) * top >= (1ll << 31) || top * den >= (1ll << 31)) return -1;
  int sh = 0;
  while ((1ll << sh) < den) ++sh;
  return sh;
}

// Workspace bytes of the training / forward / backward entry points for `batch` positions.
int64_t train_workspace_bytes(const Shape& s, int64_t batch);

}  // namespace ntbc
