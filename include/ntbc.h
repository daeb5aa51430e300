/*
 * libntbc -- Neural Texture Block Compression (BC1/BC4) on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library.  Every entry point:
 *   - takes plain pointers and sizes (no C++ or framework types);
 *   - takes DEVICE pointers for every array (caller-owned; the library never frees them) unless the
 *     argument is documented as a host struct;
 *   - is asynchronous on the HIP stream passed as `stream` (a hipStream_t, NULL = the null stream):
 *     it validates its arguments on the host, enqueues kernels and returns without synchronising;
 *   - returns NTBC_OK (0) or a negative status; on error nothing has been enqueued (argument errors)
 *     or the HIP error is reported (NTBC_EHIP) and ntbc_last_error() describes it;
 *   - allocates no device memory: scratch comes from the caller's `workspace` (size from
 *     ntbc_workspace_size) where an entry point has one.
 *
 * Data layouts
 *   Textures   row-major uint8, `row_pitch` bytes between rows; BC1 textures have 3 channels (RGB),
 *              BC4 textures 1.  Width and height are multiples of 4.
 *   Blocks     uint64 little-endian BC words, row-major over the block grid: block id
 *              b = by * (width/4) + bx.  BC1: c0 = bits 0-15, c1 = bits 16-31 (RGB565, R in the top
 *              5 bits), 2-bit code of texel i = 4y+x at bit 32+2i.  BC4: e0 = bits 0-7, e1 = bits 8-15,
 *              3-bit code of texel i at bit 16+3i.
 *   Grid       level-major, then vertex j*res_l + i (j = row), then feature: res_l = base_res << l,
 *              sum_l res_l^2 vertices of n_features each.  FP32 grids hold real values; U8 grids hold
 *              codes q with value scale_l * (q - zero_l).
 *   Weights    FP32, canonical flat order W_1, b_1, W_2, b_2, ..., W_out, b_out with W_k row-major
 *              [fan_out][fan_in].  Layers: in_dim = n_levels * n_features -> hidden_width (n_hidden
 *              times, ReLU) -> head_dim (sigmoid).
 *   Heads      head_dim floats per block position: the endpoint head (per texture in order: BC1 ->
 *              R0 G0 B0 R1 G1 B1, BC4 -> e0 e1) followed by the colour head, texel-major
 *              [texel 0..15][channels of every texture in order].  Naive variant (NTBC_NAIVE): the
 *              endpoint head followed by the weight head, texel-major [texel 0..15][one weight per
 *              texture in order].
 *
 * Paper: S. Fujieda and T. Harada, "Neural Texture Block Compression" (arXiv 2407.09543).  Section
 * numbers below refer to it.
 */
#ifndef NTBC_H
#define NTBC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------------------ */
#define NTBC_OK 0
#define NTBC_EINVAL (-1)          /* null pointer, bad size, bad enum, dims not multiples of 4     */
#define NTBC_EUNSUPPORTED (-2)    /* a valid combination this build does not implement            */
#define NTBC_EHIP (-3)            /* a HIP runtime error; see ntbc_last_error()                    */
#define NTBC_ENONFINITE (-4)      /* a training step saw a non-finite loss or gradient and left the
                                     parameters and moments untouched (ntbc_train_status)             */
#define NTBC_ENOWORKSPACE (-5)    /* workspace NULL or smaller than ntbc_workspace_size()          */

/* ---- enums ------------------------------------------------------------------------------------- */
/* The value sets below travel as int32_t (struct fields and arguments), not as C enums, so that their
 * width and the struct layouts are the same for every compiler; these names label them. */
typedef int32_t ntbc_format;     /* NTBC_BC1, NTBC_BC4                                              */
typedef int32_t ntbc_precision;  /* NTBC_FP32, NTBC_BF16, NTBC_FP8_E4M3, NTBC_FP16                  */
typedef int32_t ntbc_grid_dtype; /* NTBC_GRID_F32, NTBC_GRID_U8                                     */

#define NTBC_BC1 1
#define NTBC_BC4 4

#define NTBC_FP32 0               /* MLP in FP32 (FP32 matrix cores), FP32 accumulation             */
#define NTBC_BF16 1               /* MLP weights and layer inputs in BF16, FP32 accumulation         */
#define NTBC_FP8_E4M3 2           /* middle hidden layers in FP8 E4M3 (OCP) with per-layer power-of-two
                                     scales (ntbc_fp8_calibrate); the first layer and the head in
                                     BF16; FP32 accumulation                                         */
#define NTBC_FP16 3               /* MLP weights and layer inputs in IEEE half, FP32 accumulation    */

#define NTBC_GRID_F32 0
#define NTBC_GRID_U8 1

#define NTBC_MAX_TEXTURES 8
#define NTBC_MAX_LEVELS 12

/* Model variants (ntbc_model_desc.variant). */
#define NTBC_NTBC 0               /* Sec. 3.2: endpoint head + colour head; each texel takes the palette
                                     entry nearest to its predicted colour (Eq. dist)                 */
#define NTBC_NAIVE 1              /* Sec. 3.1, the naive approach: endpoint head + weight head; each
                                     texel takes the quantised weight w_n nearest to its predicted
                                     weight (float32 decision, ties to the smaller n): BC1 n/3, with
                                     1 - w when the endpoints are swapped into four-colour order; BC4
                                     n/7 (e0 > e1) or (n-1)/5 for n = 1..6 (the interpolated entries).
                                     Trained in two stages (ntbc_hparams.stage2_from)                 */

/* One material's model shape (host struct; sizes only). */
typedef struct {
  int32_t n_levels;       /* grid levels L, 1..NTBC_MAX_LEVELS                                      */
  int32_t base_res;       /* res_0 >= 2; res_l = base_res << l                                       */
  int32_t n_features;     /* F per level: 1, 2, 4, 8 or 16                                           */
  int32_t grid_dtype;     /* NTBC_GRID_F32 or NTBC_GRID_U8 (inference input only)                   */
  int32_t hidden_width;   /* multiple of 32, 32..256                                                 */
  int32_t n_hidden;       /* hidden layers, 1..4                                                      */
  int32_t n_textures;     /* 1..NTBC_MAX_TEXTURES                                                    */
  int32_t formats[NTBC_MAX_TEXTURES]; /* NTBC_BC1 or NTBC_BC4 per texture, in head order            */
  int32_t blocks_w;       /* block grid = texture size / 4                                           */
  int32_t blocks_h;
  int32_t variant;        /* NTBC_NTBC (0) or NTBC_NAIVE: head_dim = 6*nBC1 + 2*nBC4 + 16*n_textures */
} ntbc_model_desc;

/* Model parameters for inference (host struct of device pointers). */
typedef struct {
  const void* grid;         /* FP32: float[V][F]; U8: uint8[V][F]                                   */
  const float* grid_scale;  /* U8 only: [n_levels] scale_l                                           */
  const int32_t* grid_zero; /* U8 only: [n_levels] zero point z_l in 0..255                          */
  const float* weights;     /* FP32 canonical flat layout                                            */
  const float* fp8_scales;  /* FP8 only: [n_layers][2] = (s_x, s_w) per layer: the layer input is
                               rounded to E4M3 as x/s_x, the weight as W*(1/s_w)                      */
  int32_t flags;            /* NTBC_REUSE_PACKED: the workspace already holds the packed weights of
                               these same weights and precision from an earlier call; skip packing */
} ntbc_params;

#define NTBC_REUSE_PACKED 1

/* Message describing the last error returned on the calling host thread ("" if none).  The string
 * is owned by the library and valid until the next failing call on the same thread. */
const char* ntbc_last_error(void);

/* ---- sizes -------------------------------------------------------------------------------------- */

/* Number of FP32 values in the canonical weight layout of `d`; head_dim = 6*nBC1 + 2*nBC4 +
 * 16*(3*nBC1 + nBC4) (NTBC_NAIVE: 6*nBC1 + 2*nBC4 + 16*n_textures); grid vertex count sum_l res_l^2.
 * Host only.  Returns NTBC_EINVAL on a bad desc. */
int ntbc_model_sizes(const ntbc_model_desc* d, int64_t* n_weights, int32_t* head_dim,
                     int64_t* grid_vertices);

/* Workspace bytes needed by ntbc_infer_blocks (batch = 0), ntbc_forward / ntbc_backward and
 * ntbc_train_step for `batch` block positions at `precision`.  Host only. */
int ntbc_workspace_size(const ntbc_model_desc* d, int32_t precision, int64_t batch, size_t* bytes);

/* ---- BC format ---------------------------------------------------------------------------------- */

/* Reference encoder (Sec. 3.2 and Sec. 4.1: the reference blocks that are the training targets;
 * also the fallback).  The encoding is the project's integer REF-BC1 / REF-BC4 algorithm (two
 * candidates, exact nearest-code selection, two least-squares refinement steps in exact integer
 * arithmetic; BC1 blocks of one colour also try the optimal single-colour endpoints, whose 2/3 point
 * is the nearest value any BC1 palette entry can take in each channel), bit-reproducible.  texels: uint8 texture (3 channels for BC1, 1 for BC4), `row_pitch`
 * bytes per row.  blocks_out: uint64[(height/4)*(width/4)].  Optional sse_out (may be NULL): int32
 * per block, integer squared error of the decoded block against the texels. */
int ntbc_bc_encode_ref(const uint8_t* texels, int32_t width, int32_t height, int32_t row_pitch,
                       int32_t format, uint64_t* blocks_out, int32_t* sse_out, void* stream);

/* Decoder (Sec. 1 and Sec. 2.1; Eq. palette): BC1 four-colour mode (c0 > c1) and three-colour mode
 * (c0 <= c1: midpoint rounded half up, code 3 = black), BC4 eight-value (e0 > e1) and six-value mode
 * (codes 6, 7 = 0, 255).  Endpoints expand 565 -> 888 by bit replication; interpolants are rounded to
 * the nearest integer.  texels_out: uint8 texture with `row_pitch` bytes per row. */
int ntbc_bc_decode(const uint64_t* blocks, int32_t width, int32_t height, int32_t format,
                   uint8_t* texels_out, int32_t row_pitch, void* stream);

/* Block-major copy of a texture (the training targets' block_texels): blocks_out[(b * 16 + i) * channels
 * + c] = channel c of texel i = 4y + x of block b = by * (width/4) + bx, i.e. texel (4bx + x, 4by + y);
 * channels 3 for NTBC_BC1, 1 for NTBC_BC4.  blocks_out: uint8[(width/4)*(height/4)*16*channels]. */
int ntbc_texels_to_blocks(const uint8_t* texels, int32_t width, int32_t height, int32_t row_pitch,
                          int32_t format, uint8_t* blocks_out, void* stream);

/* Per-block integer squared error between decoded `blocks` and `texels` -> sse_out int32[n blocks]. */
int ntbc_block_sse(const uint64_t* blocks, const uint8_t* texels, int32_t width, int32_t height,
                   int32_t row_pitch, int32_t format, int32_t* sse_out, void* stream);

/* Per-block judge and fallback (Sec. 4.3: standard BC remains available for what NTBC compresses
 * badly, applied here per block): out[b] = (sse_ntbc[b] > kappa * sse_ref[b] + delta) ? ref[b] :
 * ntbc[b]; the number of replaced blocks is added to *n_fallback (device int32).  `out` may alias
 * `ntbc`. */
int ntbc_fallback(const uint64_t* ntbc, const uint64_t* ref, const int32_t* sse_ntbc,
                  const int32_t* sse_ref, int64_t n_blocks, float kappa, float delta, uint64_t* out,
                  int32_t* n_fallback, void* stream);

/* ---- inference ---------------------------------------------------------------------------------- */

/* NTBC inference (Sec. 3.2, Fig. NTBC inference; Eq. palette, Eq. dist) for block positions
 * [first_block, first_block + n_blocks): block coordinate -> bilinear lookups in every grid level ->
 * MLP (`precision`) -> sigmoid heads -> endpoints quantised as floor(y*(2^b-1)+1/2) (b = 5/6/5 or 8)
 * -> palette of the stored endpoints -> per texel the palette entry nearest to the predicted colour
 * (ties: smallest weight index) -> packed words.  BC1 endpoints are swapped when c0 < c1; equal
 * endpoints give all-zero codes.  BC4's mode follows the stored endpoint order.
 * blocks_out: uint64[n_textures][n_blocks].  heads_out (optional, may be NULL): float
 * [n_blocks][head_dim] sigmoid outputs.  workspace: >= ntbc_workspace_size(d, precision, 0).
 * Precisions: NTBC_FP32, NTBC_BF16, NTBC_FP16, and NTBC_FP8_E4M3 with p->fp8_scales set (from
 * ntbc_fp8_calibrate; FP8 needs head_dim <= 192, in_dim <= 64 and two hidden layers, else
 * NTBC_EUNSUPPORTED; its first layer and head take BF16 operands, the layers between them E4M3). */
int ntbc_infer_blocks(const ntbc_model_desc* d, const ntbc_params* p, int32_t precision,
                      int64_t first_block, int64_t n_blocks, uint64_t* blocks_out, float* heads_out,
                      void* workspace, size_t workspace_bytes, void* stream);

/* ntbc_infer_blocks for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same computation and the same output, with the
 * packed weights kept in a static device array of the library (4 MiB per GPU, held by every GPU the
 * library runs on until the process ends; every model shape the library accepts fits, the largest
 * needing 1.8 MB) instead of a caller workspace.  The calling thread's current
 * device must be the device of `stream`; its scratch address is looked up on the first call on that
 * device.  No hipMalloc, hipFree or other allocating routine is called.  Every call on one GPU shares
 * that GPU's scratch, which keeps the last call's packed weights: calls that overlap on one GPU (on
 * different streams, or from several host threads) race and must be serialised by the caller;
 * p->flags & NTBC_REUSE_PACKED is valid only when the previous call on the device packed the same
 * weights at the same precision.  Errors: as ntbc_infer_blocks, and NTBC_ENOWORKSPACE when the model's
 * packed weights (ntbc_workspace_size(d, precision, 0)) exceed the scratch. */
int ntbc_infer_blocks_noalloc(const ntbc_model_desc* d, const ntbc_params* p, int32_t precision,
                              int64_t first_block, int64_t n_blocks, uint64_t* blocks_out, float* heads_out,
                              void* stream);

/* FP8 E4M3 scales for ntbc_infer_blocks at NTBC_FP8_E4M3 (the paper has no FP8 path; per-layer,
 * per-tensor scaling as this library defines it): for every layer, s_w = the smallest power of two
 * with max|W| / s_w <= 448 (the largest finite E4M3 value; biases stay FP32) and s_x = the same for
 * the largest |input| of the layer over a calibration sample — blocks i * stride, i < min(n_sample,
 * n_positions), stride = max(1, n_positions / n_sample) — evaluated by the FP32 inference path.
 * Powers of two make the scaling exact and keep every scaled value inside the E4M3 range.
 * scales_out: device float[n_layers][2] = (s_x, s_w).  workspace: >= ntbc_workspace_size(d,
 * NTBC_FP8_E4M3, 0).  Errors: NTBC_EINVAL (NULL pointers, n_sample < 1), NTBC_ENOWORKSPACE. */
int ntbc_fp8_calibrate(const ntbc_model_desc* d, const ntbc_params* p, int64_t n_sample, float* scales_out,
                       void* workspace, size_t workspace_bytes, void* stream);

/* ---- batched decode ----------------------------------------------------------------------------- */

/* One block range of one model (a material, or one mip level of it: a mip is the same network queried
 * at the block centres of its own block grid, desc.blocks_w x desc.blocks_h). */
typedef struct {
  ntbc_model_desc desc;
  ntbc_params params;       /* device pointers; flags ignored */
  int64_t first_block, n_blocks;
  uint64_t* blocks_out;     /* device uint64[n_textures][n_blocks] */
  int32_t model_id;         /* items with equal model_id share weights and layer shapes: one packed copy */
} ntbc_batch_item;

/* Bytes of the host table that ntbc_batch_plan fills for n_items items.  Host only. */
int ntbc_batch_table_size(int32_t n_items, size_t* bytes);

/* Plans the load-time decode of many block ranges at `precision` (NTBC_BF16, NTBC_FP16 or
 * NTBC_FP8_E4M3 with params.fp8_scales): one launch per kernel instance (hidden width, first-layer
 * K-steps), items grouped by instance.  Writes a table image into `table` (host memory,
 * >= ntbc_batch_table_size) that embeds device addresses inside `workspace` (device memory of
 * *workspace_bytes; pass NULL first to learn the size, then plan again with the workspace).  The
 * caller copies the table to device memory for ntbc_infer_batch.  Host only.  Errors: NTBC_EINVAL,
 * NTBC_EUNSUPPORTED (shapes the fused kernel does not take). */
int ntbc_batch_plan(const ntbc_batch_item* items, int32_t n_items, int32_t precision, void* workspace, void* table,
                    size_t table_bytes, size_t* workspace_bytes);

/* Packs every distinct model's weights into the workspace (once; again after the weights change). */
int ntbc_batch_pack(const void* table, void* workspace, size_t workspace_bytes, void* stream);

/* The kernel instances of a plan (one launch each): n_groups receives their count and, when groups_out
 * is not NULL, groups_out[8 g .. 8 g + 7] = precision, hidden width, first-layer K-steps, unrolled
 * middle layers (-1: a run-time count), BC1 and BC4 textures of the register epilogue (-1: heads staged
 * in LDS), tile waves, items, for g < min(*n_groups, max_groups).  Host only. */
int ntbc_batch_groups(const void* table, int32_t* groups_out, int32_t max_groups, int32_t* n_groups);

/* Tile shape of one kernel instance of a plan: `waves` (2, 4 or 8) waves of 32 block positions per
 * workgroup (4 after ntbc_batch_plan; 2 and 8 exist for BF16 only, else NTBC_EUNSUPPORTED; a shape
 * whose LDS does not fit returns NTBC_EINVAL).  Rewrites the host table; the caller copies it to its
 * device copy again before ntbc_infer_batch.  The blocks do not depend on the shape.  Host only.  This
 * is what the tile autotuner (paper_2407_09543_amd.autotune) times. */
int ntbc_batch_set_waves(void* table, int32_t group, int32_t waves);

/* Decodes every item of a plan: `table` is the host image, `table_device` the caller's device copy of
 * it.  stamps (optional, device uint64[n_items + 1]): [0] = the real-time counter (100 MHz) when the
 * batch starts, [1 + i] = when item i's last tile finished.  Stream-ordered and allocation-free, so a
 * caller may capture it in a HIP graph and replay it. */
int ntbc_infer_batch(const void* table, const void* table_device, void* workspace, size_t workspace_bytes,
                     uint64_t* stamps, void* stream);

/* ---- the paper's own network layout -------------------------------------------------------------- */

/* One model of the paper's layout (Sec. 3.4; Sec. 4.1 for the material layouts): an endpoint network on
 * the block's cell of a multi-resolution grid and a colour network on each texel's cell of a second
 * grid, both with 2 features per level, three hidden layers of 64 SELU units (lambda =
 * 1.0507009873554805, alpha = 1.6732632423543772) and sigmoid outputs, evaluated with IEEE-half
 * operands and FP32 accumulation.  A block's endpoints come from one endpoint-network run and its 16
 * texels' predicted colours from 16 colour-network runs; the heads are assembled in the NTBC layout
 * and packed as ntbc_infer_blocks packs them (Eq. dist).  The aggressive layout is one model over
 * every texture; the conservative layout is two models (the BC1 textures, the BC4 textures), i.e. two
 * calls.  Host struct, sizes only. */
typedef struct {
  int32_t ep_levels, ep_base_res;     /* endpoint grid: levels 1..8, coarsest resolution (paper: 7, 16) */
  int32_t col_levels, col_base_res;   /* colour grid over texel cells (paper: 8, 16)                    */
  int32_t grid_dtype;                 /* NTBC_GRID_F32 or NTBC_GRID_U8 (both grids)                     */
  int32_t n_textures;
  int32_t formats[NTBC_MAX_TEXTURES]; /* endpoint outputs 6*nBC1 + 2*nBC4 <= 64, colour outputs
                                         3*nBC1 + nBC4 <= 32, per texture in order                      */
  int32_t blocks_w, blocks_h;         /* block grid; the colour grid's cells are the 4*blocks texels   */
} ntbc_faithful_desc;

/* Parameters (host struct of device pointers).  Grids level-major, vertex j*res + i, 2 features;
 * U8 grids with per-level scale and zero point.  Weights in the canonical FP32 layout of each network:
 * W1,b1,W2,b2,W3,b3,W4,b4 with W row-major [out][in]; in = 2*levels, hidden 64, out as above. */
typedef struct {
  const void* ep_grid;
  const float* ep_scale;
  const int32_t* ep_zero;
  const void* col_grid;
  const float* col_scale;
  const int32_t* col_zero;
  const float* ep_weights;
  const float* col_weights;
} ntbc_faithful_params;

/* FP32 weights of each network and the workspace bytes of ntbc_faithful_infer.  Host only. */
int ntbc_faithful_sizes(const ntbc_faithful_desc* d, int64_t* ep_weights, int64_t* col_weights,
                        size_t* workspace_bytes);

/* Blocks [first_block, first_block + n_blocks) of every texture of the model: blocks_out
 * uint64[n_textures][n_blocks]; heads_out (optional, NULL to skip) float[n_blocks][E + 16*C] in the
 * NTBC head layout.  Packs the weights into the workspace on every call.  Errors: NTBC_EINVAL,
 * NTBC_ENOWORKSPACE. */
int ntbc_faithful_infer(const ntbc_faithful_desc* d, const ntbc_faithful_params* p, int64_t first_block,
                        int64_t n_blocks, uint64_t* blocks_out, float* heads_out, void* workspace,
                        size_t workspace_bytes, void* stream);

/* ---- training ----------------------------------------------------------------------------------- */

/* Training state (host struct of device pointers, caller-owned).  Master parameters in FP32; Adam
 * moments of the same shapes (zero before the first step); gradient buffers overwritten by each step. */
typedef struct {
  float* grid;        /* [V][F] master grid                                                            */
  float* weights;     /* [n_weights] master weights, canonical layout                                  */
  float* m_grid;      /* Adam first moments                                                            */
  float* v_grid;      /* Adam second moments                                                           */
  float* m_weights;
  float* v_weights;
  float* d_grid;      /* gradient of the last step                                                     */
  float* d_weights;
} ntbc_train_state;

/* Training targets (host struct of device pointers): the reference blocks and the textures. */
typedef struct {
  const uint64_t* ref_blocks;                 /* [n_textures][n_positions] reference BC words          */
  const uint8_t* texels[NTBC_MAX_TEXTURES];   /* per texture, row-major, tightly packed (pitch =
                                                 4*blocks_w*channels)                                   */
  const uint8_t* block_texels[NTBC_MAX_TEXTURES]; /* optional (NULL): the same texels block-major, as
                                                 ntbc_texels_to_blocks writes them; when set for every
                                                 texture the losses read these (a block's 16 texels
                                                 are one contiguous run) instead of `texels`         */
} ntbc_targets;

/* Hyper-parameters (host struct).  Paper Sec. 3.4: Adam beta1 0.9, beta2 0.999, eps 1e-15; learning
 * rates 0.01 (grid) and 0.005 (MLP); 10 warm-up steps then cosine annealing to 0 at total_steps;
 * T = 0.01.  Sec. 3.3: qat = 1 fake-quantises every grid level to 8 bits with its current min/max (the range
 * widened to contain 0, as for ntbc_quantize_grid). */
typedef struct {
  float lr_grid, lr_mlp;
  float beta1, beta2, eps;
  float temperature;
  int32_t warmup, total_steps;
  int32_t qat;
  int32_t precision;        /* NTBC_FP32, or NTBC_BF16: the MLP products (forward, dX and dW) take
                               bfloat16 operands on the matrix cores with FP32 accumulation; master
                               parameters, losses, grid scatter and Adam stay FP32                   */
  float loss_weights[4];    /* weights of L_e, L_c, L_cd(endpoint), L_cd(colour) in the gradient; 1 = paper */
  int32_t deterministic;    /* 0: the grid scatter (and, for shapes outside the fused bfloat16 path, the
                               split weight products) add with FP32 atomics, so the gradients depend on
                               their order in the last bits.  1: bitwise repeatable parameters: the grid
                               gradient is summed as 64-bit fixed-point integers at a per-step power-of-two
                               scale 2^(61 - ceil(log2(batch * max|dX|))) (order-independent; each term
                               rounded to that scale, which is far finer than FP32's resolution of the
                               sums) and every weight product runs unsplit.  The reported losses are
                               FP32 atomic sums in both modes. */
  int32_t stage2_from;      /* NTBC_NAIVE only (Sec. 3.1): steps >= stage2_from are the second stage, which
                               decodes with the quantised weights w_n (the gradient reaches the endpoints
                               only) and updates only the endpoint head's rows of the last layer's weights
                               and biases; the grid, the hidden layers and the weight head keep their
                               values and moments.  The paper's split is the first 80% of the steps. */
} ntbc_hparams;

/* Block ids passed to the training entry points are clamped into [0, blocks_w*blocks_h). */

/* Training precision (ntbc_forward, ntbc_backward, ntbc_hparams.precision): NTBC_FP32 or NTBC_BF16
 * (bfloat16 operands of the MLP products, FP32 accumulation); others return NTBC_EUNSUPPORTED. */

/* Forward pass for a batch (paper Sec. 3.2, Fig. NTBC training, network part): the sigmoid heads of
 * block positions ids[0..n) from the FP32 master grid (fake-quantised per level when qat = 1: Sec. 3.3,
 * Eq. quantizer with s, z from the level's min/max) and FP32 weights.  heads_out: float[n][head_dim].
 * Nothing is kept for the backward pass; ntbc_backward recomputes the activations. */
int ntbc_forward(const ntbc_model_desc* d, const float* grid, const float* weights, int32_t qat,
                 int32_t precision, const int32_t* ids, int32_t n, float* heads_out, void* workspace,
                 size_t workspace_bytes, void* stream);

/* Backward pass (Sec. 3.2, Fig. NTBC training: the network and the feature grids are learned jointly
 * by backpropagation; Sec. 2.3 and Sec. 3.3: the quantiser's straight-through estimator under QAT):
 * given dL/d(heads) for the same batch, recomputes the forward activations and ADDS the gradients to
 * d_grid ([V][F], scatter through the bilinear weights; with qat = 1 the quantiser's straight-through
 * pass-through: 1 inside the level's range, 0 where clamped) and d_weights (canonical layout).  The
 * caller zeroes them first. */
int ntbc_backward(const ntbc_model_desc* d, const float* grid, const float* weights, int32_t qat,
                  int32_t precision, const int32_t* ids, int32_t n, const float* d_heads, float* d_grid,
                  float* d_weights, void* workspace, size_t workspace_bytes, void* stream);

/* NTBC loss (Sec. 3.2, Eqs. lossNTBC; App. A): for heads of block positions ids, losses_out[0..3] =
 * L_e, L_c, L_cd(endpoint branch), L_cd(colour branch), each a mean over its elements; d_heads_out =
 * dL/d(heads) of loss_weights . losses, with the argmax of the decoded-colour terms differentiated as
 * the softmax(d/T) expectation of the reference palette (straight-through).  losses_out (device
 * float[5]) is overwritten; losses_out[4] = 1 if a head or gradient was not finite. */
int ntbc_loss_grad(const ntbc_model_desc* d, const ntbc_targets* t, const float* heads, const int32_t* ids,
                   int32_t n, float temperature, const float* loss_weights, float* losses_out,
                   float* d_heads_out, void* stream);

/* Naive-approach loss (Sec. 3.1; d->variant = NTBC_NAIVE): decoded colours x = (1 - w) e0^ + w e1^ per
 * texel and channel from the predicted endpoints and weights of heads ([n][head_dim]); stage 1 takes
 * the continuous weight w, stage 2 the nearest quantised weight w_n of the block's mode (BC4: eight
 * values when e0^ > e1^; the endpoints stay continuous and unswapped).  losses_out[0] = L = the mean of
 * (x - c)^2 over n * 16 texels * the channels of every texture, losses_out[1..3] = 0, losses_out[4] = 1
 * if a head or gradient was not finite (device float[5], overwritten).  d_heads_out = dL/d(heads)
 * (stage 2: zero on the weight head).  Errors: NTBC_EINVAL (stage not 1 or 2, d->variant not naive). */
int ntbc_naive_loss_grad(const ntbc_model_desc* d, const ntbc_targets* t, const float* heads, const int32_t* ids,
                         int32_t n, int32_t stage, float* losses_out, float* d_heads_out, void* stream);

/* One training iteration (Sec. 3.2 training procedure and Eqs. lossNTBC; App. A straight-through
 * estimator; Sec. 3.3 QAT; Sec. 3.4 Adam, learning rates, warm-up and cosine annealing): forward, loss,
 * backward, then dense Adam on grid and weights with the learning rates of step `step` (0-based) of the
 * schedule.  losses_out (device float[5]) receives the
 * four losses and the skip flag: when a non-finite value is seen the parameters and moments are left
 * untouched and losses_out[4] = 1.  batch_ids: device int32[batch] block positions.  NTBC_NAIVE models
 * train with ntbc_naive_loss_grad's loss instead (Sec. 3.1), stage 2 from step h->stage2_from on. */
int ntbc_train_step(const ntbc_model_desc* d, const ntbc_train_state* st, const ntbc_targets* t,
                    const int32_t* batch_ids, int32_t batch, int64_t step, const ntbc_hparams* h,
                    float* losses_out, void* workspace, size_t workspace_bytes, void* stream);

/* Outcome of a training step, for callers that want it as a status code: waits for `stream` (the
 * only synchronising call of the library), reads the skip flag losses_out[4] that ntbc_train_step
 * wrote on that stream (`losses` = the step's device losses_out) and returns NTBC_ENONFINITE when the
 * step saw a non-finite loss or gradient (the parameters and Adam moments were left untouched, Sec.
 * 3.4's update skipped), NTBC_OK otherwise.  The step itself stays asynchronous: a caller may also read
 * the flag later, or never. */
int ntbc_train_status(const float* losses, void* stream);

/* ---- the paper's own layout: training ------------------------------------------------------------ */

/* Training state of one model of the paper's layout (host struct of device pointers, caller-owned):
 * FP32 master grids ([V][2], level-major as in ntbc_faithful_params) and weights (each network's
 * canonical layout, sizes from ntbc_faithful_sizes), Adam moments of the same shapes (zero before the
 * first step) and the gradient buffers that each step overwrites. */
typedef struct {
  float *ep_grid, *col_grid, *ep_weights, *col_weights;
  float *m_ep_grid, *v_ep_grid, *m_col_grid, *v_col_grid;
  float *m_ep_weights, *v_ep_weights, *m_col_weights, *v_col_weights;
  float *d_ep_grid, *d_col_grid, *d_ep_weights, *d_col_weights;
} ntbc_faithful_train_state;

/* Workspace bytes of ntbc_faithful_train_step for `batch` blocks.  Host only. */
int ntbc_faithful_train_size(const ntbc_faithful_desc* d, int32_t batch, size_t* workspace_bytes);

/* One training iteration of one model of the paper's layout (Sec. 3.2 training procedure and Eqs.
 * lossNTBC; App. A straight-through estimator; Sec. 3.3 QAT; Sec. 3.4 configuration, Adam and schedule;
 * Sec. 4.1 layouts): the endpoint network at the batch's blocks and the colour network at their 16 *
 * batch texels (FP32 products, SELU hidden layers), the heads assembled in the NTBC layout, the NTBC
 * losses and their straight-through gradient (as ntbc_loss_grad: the aggressive layout's dummy distance
 * nodes change neither), the backward through both networks into both grids (the quantiser's
 * pass-through when h->qat), then Adam on the four parameter sets (grids at lr_grid, networks at lr_mlp,
 * the learning rates of step `step` of the schedule).  d->grid_dtype must be NTBC_GRID_F32 (the master
 * grids); h->precision NTBC_FP32, else NTBC_EUNSUPPORTED; h->deterministic as for ntbc_train_step;
 * t: the targets of the model's textures, in their order.  losses_out (device float[5]) as for
 * ntbc_train_step: a non-finite value skips the update and sets losses_out[4] = 1.  A conservative
 * material trains its two models with one call each.  Errors: NTBC_EINVAL, NTBC_ENOWORKSPACE,
 * NTBC_EUNSUPPORTED. */
int ntbc_faithful_train_step(const ntbc_faithful_desc* d, const ntbc_faithful_train_state* st,
                             const ntbc_targets* t, const int32_t* batch_ids, int32_t batch, int64_t step,
                             const ntbc_hparams* h, float* losses_out, void* workspace, size_t workspace_bytes,
                             void* stream);

/* Training batch `step`: `batch` block-position ids drawn uniformly with replacement from
 * [0, n_positions) (the paper leaves the sampling unspecified).  Generator: SplitMix64 (Steele, Lea &
 * Flood 2014).  The stream key is k = mix(mix(mix(0, seed), 0xBA7C4), step) with
 * mix(h, p) = splitmix64_output((h ^ p) + 0x9E3779B97F4A7C15); draw i (0-based) is
 * z = splitmix64_output(k + (i+1) * 0x9E3779B97F4A7C15) and id = ((z >> 32) * n_positions) >> 32.
 * ids_out: device int32[batch]. */
int ntbc_batch_ids(uint64_t seed, int64_t step, int32_t batch, int64_t n_positions, int32_t* ids_out,
                   void* stream);

/* 8-bit grid for inference (Sec. 3.3): per level l, over the level's range widened to contain 0 (Sec.
 * 2.3: the zero point makes real 0 an exact code) lo = min(min, 0), hi = max(max, 0): s_l = (hi-lo)/255
 * and z_l = clamp(rne(-lo/s_l), 0, 255) (s = 1, z = 0 for an all-zero level), codes q = clamp(rne(g/s_l)
 * + z_l, 0, 255); all in float32.  The same (s, z) drive the fake quantisation of training (qat = 1).
 * codes: uint8[V][F]; scale: float[n_levels]; zero: int32[n_levels]. */
int ntbc_quantize_grid(const ntbc_model_desc* d, const float* grid, uint8_t* codes, float* scale,
                       int32_t* zero, void* workspace, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NTBC_H */
