// Host-side parts of the C ABI: error reporting, model-shape validation and sizes.
#include <cstring>

#include "common.h"

namespace ntbc {

static thread_local char g_last_error[512] = "";

int fail(int status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return status;
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(NTBC_EHIP, "%s: launch failed: %s", what, hipGetErrorString(e));
  return NTBC_OK;
}

int make_shape(const ntbc_model_desc* d, Shape* s) {
  NTBC_REQUIRE(d != nullptr, "model desc is NULL");
  NTBC_REQUIRE(d->n_levels >= 1 && d->n_levels <= NTBC_MAX_LEVELS, "n_levels %d out of 1..%d",
               d->n_levels, NTBC_MAX_LEVELS);
  NTBC_REQUIRE(d->base_res >= 2 && d->base_res <= 65536, "base_res %d must be >= 2", d->base_res);
  NTBC_REQUIRE(d->n_features == 1 || d->n_features == 2 || d->n_features == 4 ||
                   d->n_features == 8 || d->n_features == 16,
               "n_features %d must be 1, 2, 4, 8 or 16", d->n_features);
  NTBC_REQUIRE(d->grid_dtype == NTBC_GRID_F32 || d->grid_dtype == NTBC_GRID_U8, "bad grid_dtype %d",
               d->grid_dtype);
  NTBC_REQUIRE(d->hidden_width >= 32 && d->hidden_width <= 256 && d->hidden_width % 32 == 0,
               "hidden_width %d must be a multiple of 32 in 32..256", d->hidden_width);
  NTBC_REQUIRE(d->n_hidden >= 1 && d->n_hidden <= 4, "n_hidden %d out of 1..4", d->n_hidden);
  NTBC_REQUIRE(d->n_textures >= 1 && d->n_textures <= NTBC_MAX_TEXTURES, "n_textures %d out of 1..%d",
               d->n_textures, NTBC_MAX_TEXTURES);
  NTBC_REQUIRE(d->variant == NTBC_NTBC || d->variant == NTBC_NAIVE, "variant %d is not NTBC_NTBC or NTBC_NAIVE",
               d->variant);
  NTBC_REQUIRE(d->blocks_w >= 1 && d->blocks_h >= 1, "block grid %dx%d must be positive", d->blocks_w,
               d->blocks_h);
  const int64_t top = (int64_t)d->base_res << (d->n_levels - 1);
  NTBC_REQUIRE(top <= (1 << 15), "finest grid level %lld too large", (long long)top);
  std::memset(s, 0, sizeof(*s));
  s->n_levels = d->n_levels;
  s->base_res = d->base_res;
  s->n_features = d->n_features;
  s->in_dim = d->n_levels * d->n_features;
  NTBC_REQUIRE(s->in_dim <= 256, "in_dim %d = n_levels*n_features exceeds 256", s->in_dim);
  s->hidden = d->hidden_width;
  s->n_hidden = d->n_hidden;
  s->n_layers = d->n_hidden + 1;
  s->n_textures = d->n_textures;
  int e = 0, c = 0;
  for (int t = 0; t < d->n_textures; ++t) {
    const int f = d->formats[t];
    NTBC_REQUIRE(f == NTBC_BC1 || f == NTBC_BC4, "formats[%d] = %d is not NTBC_BC1 or NTBC_BC4", t, f);
    s->formats[t] = f;
    s->ep_off[t] = e;
    s->ch_off[t] = c;
    e += f == NTBC_BC1 ? 6 : 2;
    c += f == NTBC_BC1 ? 3 : 1;
  }
  s->endpoint_dim = e;
  s->channels = c;
  s->naive = d->variant == NTBC_NAIVE;
  s->head_dim = e + 16 * (s->naive ? d->n_textures : c);
  s->blocks_w = d->blocks_w;
  s->blocks_h = d->blocks_h;
  s->n_positions = (int64_t)d->blocks_w * d->blocks_h;
  int64_t off = 0;
  for (int l = 0; l < d->n_levels; ++l) {
    s->level_offset[l] = off;
    const int64_t r = (int64_t)d->base_res << l;
    off += r * r;
  }
  s->level_offset[d->n_levels] = off;
  s->grid_vertices = off;
  int64_t w = 0;
  for (int k = 0; k < s->n_layers; ++k) {
    s->layer_in[k] = k == 0 ? s->in_dim : s->hidden;
    s->layer_out[k] = k == s->n_layers - 1 ? s->head_dim : s->hidden;
    s->w_off[k] = w;
    w += (int64_t)s->layer_in[k] * s->layer_out[k];
    s->b_off[k] = w;
    w += s->layer_out[k];
  }
  s->n_weights = w;
  return NTBC_OK;
}

}  // namespace ntbc

extern "C" const char* ntbc_last_error(void) { return ntbc::g_last_error; }

extern "C" int ntbc_model_sizes(const ntbc_model_desc* d, int64_t* n_weights, int32_t* head_dim,
                                int64_t* grid_vertices) {
  ntbc::Shape s;
  int st = ntbc::make_shape(d, &s);
  if (st != NTBC_OK) return st;
  if (n_weights) *n_weights = s.n_weights;
  if (head_dim) *head_dim = s.head_dim;
  if (grid_vertices) *grid_vertices = s.grid_vertices;
  return NTBC_OK;
}
