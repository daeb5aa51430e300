"""BC1 / BC4 block format and the integer reference encoders (oracle; test infrastructure only).

Paper anchors: the BC1 and BC4 formats (Sec. 1 and Sec. 2.1: 8-byte blocks; BC1 = two RGB565 endpoints
and 16 two-bit indices; BC4 = two 8-bit endpoints and 16 three-bit indices, with six interpolated
values when e0 > e1 and four plus the special values 0 and 1 otherwise), the palette (Sec. 3,
Eq. palette) and the BC4 weights of the six-value mode (Sec. 3, Eq. weightBC4).

Readings where the paper is silent (each also listed in the design notes of the repository):
  * Word layout: little-endian 64-bit words.  BC1: c0 in bits 0-15, c1 in bits 16-31, the 2-bit code of
    texel i = 4y+x at bit 32+2i.  BC4: e0 in bits 0-7, e1 in bits 8-15, the 3-bit code of texel i at
    bit 16+3i.  RGB565 puts R in bits 15-11, G in 10-5, B in 4-0.
  * 5/6-bit endpoints expand to 8 bits by bit replication.
  * Interpolated palette entries are the real-valued Eq. palette rounded to the nearest integer
    (thirds, fifths and sevenths of integers never tie; BC1's three-colour midpoint rounds halves up).
  * BC1 with c0 <= c1 is the three-colour mode: code 2 is the midpoint and code 3 decodes to black.
  * "Logical" index n is the paper's weight order (w_n increasing from e0 to e1, Eq. palette and
    Eq. weightBC4); the stored code of the format differs (endpoints are codes 0 and 1).
  * Ties between palette entries go to the smallest logical index.

The reference encoders (REF-BC1, REF-BC4) stand in for the third-party encoder the paper uses to make
its training targets (Sec. 3.2 and Sec. 4.1, "two refine steps").  They are defined here step by step
in exact integer arithmetic, so that any implementation can match them bit for bit:

REF-BC1, per block of texels p_i (i = 0..15, 8-bit RGB):
  1. Candidate A: the two texels farthest apart (integer squared distance); ties go to the
     lexicographically smallest pair (i, j), i < j.
  2. Candidate B: per-channel bounding box inset by (max-min)>>4 (van Waveren, "Real-Time DXT
     Compression", 2006).  The channel with the largest range (ties: lowest channel) is the main axis;
     another channel's lo/hi are swapped when its integer covariance with the main channel,
     16*sum(p_c p_m) - sum(p_c) sum(p_m), is negative.  Endpoint 0 takes the (possibly swapped) highs.
  3. Each candidate endpoint quantises to RGB565 by q5 = (31v+127)//255, q6 = (63v+127)//255 (the
     exact nearest code; no ties exist).
  4. Canonical order: c0 = pack565(end0), c1 = pack565(end1), swapped if c0 < c1 so the block is in
     four-colour mode; if c0 == c1 every code is 0.
  5. Each texel takes the palette entry of least integer squared error (ties: smallest logical n).
  6. The candidate with the smaller block SSE is kept (ties: A).
  7. Two least-squares refinement steps.  From the logical indices k_i the endpoints that minimise
     sum_i ((3-k_i) a + k_i b - 3 p_i)^2 per channel are a = 3(Sbb Sap - Sab Sbp)/D and
     b = 3(Saa Sbp - Sab Sap)/D with D = Saa Sbb - Sab^2 (alpha_i = 3-k_i, beta_i = k_i).  They are
     rounded to 5/6 bits as round-half-up of (num/D)*31/255 (resp. 63/255) after clamping num to
     [0, 255 D]; steps 4-5 are redone, and the result is kept only if the block SSE strictly falls.
     D = 0 skips the step.
  8. A block whose 16 texels are one colour (r, g, b) also tries the optimal single-colour endpoints:
     per channel, from a table over the 256 values, the code pair (a, b) (5 bits for R and B, 6 for G)
     whose four-colour 2/3 point (2 E(a) + E(b) + 1) // 3 (E = bit replication) is nearest to the
     value, ties to the smallest a, then the smallest b; every palette entry of every BC1 block is such
     a point, so the per-channel error is the least any block can reach.  Steps 4-5 are redone with
     q0 = (a_r, a_g, a_b), q1 = (b_r, b_g, b_b), and the result is kept if the block SSE strictly falls.
REF-BC4, per block of 8-bit values v_i:
  1. Candidate 8: e0 = max, e1 = min (e0 == e1 makes it the six-value mode with every texel on e0).
  2. Candidate 6: e0 = min, e1 = max over texels other than 0 and 255 (none: e0 = e1 = 0).
  3. Codes by least squared error (ties: smallest logical n).
  4. Two least-squares refinement steps per candidate, in sevenths (eight-value mode, all texels) or
     fifths (six-value mode, texels on the special values 0/255 excluded); endpoints rounded half up
     after clamping to [0, 255]; a step that leaves its mode (e0 > e1 for eight-value, e0 <= e1 for
     six-value) or does not strictly lower the SSE is dropped.
  5. The smaller SSE wins (ties: candidate 8).
"""
from __future__ import annotations

import numpy as np

# logical index n (weight order) -> stored code
BC1_CODE_OF_LOGICAL = np.array([0, 2, 3, 1], dtype=np.int64)
BC4_CODE_OF_LOGICAL_8 = np.array([0, 2, 3, 4, 5, 6, 7, 1], dtype=np.int64)
BC4_CODE_OF_LOGICAL_6 = np.array([6, 0, 2, 3, 4, 5, 1, 7], dtype=np.int64)


# ------------------------------------------------------------------------------------------------
# RGB565
# ------------------------------------------------------------------------------------------------
def unpack565(c):
    c = np.asarray(c, dtype=np.int64)
    return (c >> 11) & 31, (c >> 5) & 63, c & 31


def pack565(r, g, b):
    return (np.asarray(r, np.int64) << 11) | (np.asarray(g, np.int64) << 5) | np.asarray(b, np.int64)


def expand5(v):
    v = np.asarray(v, dtype=np.int64)
    return (v << 3) | (v >> 2)


def expand6(v):
    v = np.asarray(v, dtype=np.int64)
    return (v << 2) | (v >> 4)


def endpoint_rgb8(c):
    """RGB565 code(s) -> 8-bit RGB by bit replication, [..., 3] int64."""
    r, g, b = unpack565(c)
    return np.stack([expand5(r), expand6(g), expand5(b)], axis=-1)


def quant565(rgb8):
    """8-bit RGB [..., 3] -> nearest 5/6/5-bit codes [..., 3]."""
    v = np.asarray(rgb8, dtype=np.int64)
    return np.stack([(v[..., 0] * 31 + 127) // 255, (v[..., 1] * 63 + 127) // 255,
                     (v[..., 2] * 31 + 127) // 255], axis=-1)


# ------------------------------------------------------------------------------------------------
# BC1
# ------------------------------------------------------------------------------------------------
def bc1_palette(c0, c1):
    """Decoded palette [..., 4 codes, 3] int64 of BC1 blocks with endpoint codes c0, c1."""
    c0 = np.asarray(c0, dtype=np.int64)
    c1 = np.asarray(c1, dtype=np.int64)
    e0 = endpoint_rgb8(c0)
    e1 = endpoint_rgb8(c1)
    four = (c0 > c1)[..., None]
    p2 = np.where(four, (2 * e0 + e1 + 1) // 3, (e0 + e1 + 1) >> 1)
    p3 = np.where(four, (e0 + 2 * e1 + 1) // 3, 0)
    return np.stack([e0, e1, p2, p3], axis=-2)


def bc1_fields(words):
    w = np.asarray(words, dtype=np.uint64)
    c0 = (w & np.uint64(0xFFFF)).astype(np.int64)
    c1 = ((w >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.int64)
    codes = np.stack([((w >> np.uint64(32 + 2 * i)) & np.uint64(3)).astype(np.int64)
                      for i in range(16)], axis=-1)
    return c0, c1, codes


def bc1_pack(c0, c1, codes):
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    codes = np.asarray(codes, dtype=np.uint64)
    w = c0 | (c1 << np.uint64(16))
    for i in range(16):
        w = w | (codes[..., i] << np.uint64(32 + 2 * i))
    return w


def bc1_decode(words):
    """BC1 words [...] -> texels uint8 [..., 16, 3] (both the four- and three-colour modes)."""
    c0, c1, codes = bc1_fields(words)
    pal = bc1_palette(c0, c1)                                    # [..., 4, 3]
    out = np.take_along_axis(pal, codes[..., :, None], axis=-2)  # [..., 16, 3]
    return out.astype(np.uint8)


# ------------------------------------------------------------------------------------------------
# BC4
# ------------------------------------------------------------------------------------------------
def bc4_palette(e0, e1):
    """Decoded palette [..., 8 codes] int64 of BC4 blocks with endpoints e0, e1 (0..255)."""
    e0 = np.asarray(e0, dtype=np.int64)
    e1 = np.asarray(e1, dtype=np.int64)
    eight = e0 > e1
    cols = [e0, e1]
    for j in range(1, 7):
        v8 = ((7 - j) * e0 + j * e1 + 3) // 7
        if j <= 4:
            v6 = ((5 - j) * e0 + j * e1 + 2) // 5
        elif j == 5:
            v6 = np.zeros_like(e0)
        else:
            v6 = np.full_like(e0, 255)
        cols.append(np.where(eight, v8, v6))
    return np.stack(cols, axis=-1)


def bc4_fields(words):
    w = np.asarray(words, dtype=np.uint64)
    e0 = (w & np.uint64(0xFF)).astype(np.int64)
    e1 = ((w >> np.uint64(8)) & np.uint64(0xFF)).astype(np.int64)
    codes = np.stack([((w >> np.uint64(16 + 3 * i)) & np.uint64(7)).astype(np.int64)
                      for i in range(16)], axis=-1)
    return e0, e1, codes


def bc4_pack(e0, e1, codes):
    e0 = np.asarray(e0, dtype=np.uint64)
    e1 = np.asarray(e1, dtype=np.uint64)
    codes = np.asarray(codes, dtype=np.uint64)
    w = e0 | (e1 << np.uint64(8))
    for i in range(16):
        w = w | (codes[..., i] << np.uint64(16 + 3 * i))
    return w


def bc4_decode(words):
    """BC4 words [...] -> texels uint8 [..., 16]."""
    e0, e1, codes = bc4_fields(words)
    pal = bc4_palette(e0, e1)
    return np.take_along_axis(pal, codes, axis=-1).astype(np.uint8)


def bc4_logical_order(e0, e1):
    """[..., 8] stored code of each logical index n for the block's mode."""
    eight = (np.asarray(e0) > np.asarray(e1))[..., None]
    return np.where(eight, BC4_CODE_OF_LOGICAL_8, BC4_CODE_OF_LOGICAL_6)


# ------------------------------------------------------------------------------------------------
# Image <-> block helpers
# ------------------------------------------------------------------------------------------------
def image_to_blocks(img):
    """uint8 [H][W] or [H][W][C] -> [H/4 * W/4, 16, C] (block id = by*(W/4)+bx, texel = 4y+x)."""
    t = img if img.ndim == 3 else img[..., None]
    h, w, c = t.shape
    return t.reshape(h // 4, 4, w // 4, 4, c).transpose(0, 2, 1, 3, 4).reshape(-1, 16, c)


def blocks_to_image(blocks, height, width):
    """[H/4 * W/4, 16, C] -> [H][W][C]."""
    c = blocks.shape[-1]
    return blocks.reshape(height // 4, width // 4, 4, 4, c).transpose(0, 2, 1, 3, 4).reshape(
        height, width, c)


# ------------------------------------------------------------------------------------------------
# REF-BC1
# ------------------------------------------------------------------------------------------------
def _bc1_finish(q0, q1, p):
    """Steps 4-5 of REF-BC1 for endpoint codes q0, q1 [nb, 3] (5/6/5 bits) and texels p [nb, 16, 3].

    Returns (c0, c1, codes [nb,16], logical [nb,16], sse [nb])."""
    c0 = pack565(q0[:, 0], q0[:, 1], q0[:, 2])
    c1 = pack565(q1[:, 0], q1[:, 1], q1[:, 2])
    swap = c0 < c1
    c0, c1 = np.where(swap, c1, c0), np.where(swap, c0, c1)
    pal = bc1_palette(c0, c1)                                   # [nb, 4 codes, 3]
    lpal = pal[:, BC1_CODE_OF_LOGICAL, :]                       # [nb, 4 logical, 3]
    err = ((lpal[:, None, :, :] - p[:, :, None, :]) ** 2).sum(axis=-1)   # [nb, 16, 4]
    n = np.argmin(err, axis=2)                                  # first minimum: smallest n
    eq = c0 == c1
    n[eq] = 0
    codes = BC1_CODE_OF_LOGICAL[n]
    sse = np.take_along_axis(err, n[:, :, None], axis=2)[:, :, 0].sum(axis=1)
    return c0, c1, codes, n, sse


def _round_half_up_ratio(num, den, mul, lim):
    """round-half-up of (num/den) * mul / 255 with num clamped to [0, 255*den]; den > 0."""
    num = np.clip(num, 0, den * 255)
    return (2 * num * mul + den * 255) // (2 * den * 255)


def _bc1_refine(n, p):
    """Least-squares endpoints (step 7 of REF-BC1) from logical indices n [nb,16]."""
    a = 3 - n
    b = n
    saa = (a * a).sum(axis=1)
    sbb = (b * b).sum(axis=1)
    sab = (a * b).sum(axis=1)
    sap = (a[:, :, None] * p).sum(axis=1)                        # [nb, 3]
    sbp = (b[:, :, None] * p).sum(axis=1)
    det = saa * sbb - sab * sab
    ok = det > 0
    d = np.where(ok, det, 1)[:, None]
    num_a = 3 * (sbb[:, None] * sap - sab[:, None] * sbp)
    num_b = 3 * (saa[:, None] * sbp - sab[:, None] * sap)
    mul = np.array([31, 63, 31], dtype=np.int64)[None, :]
    qa = _round_half_up_ratio(num_a, d, mul, 255)
    qb = _round_half_up_ratio(num_b, d, mul, 255)
    return ok, qa, qb


def _select(mask, new, old):
    return tuple(np.where(mask.reshape((-1,) + (1,) * (np.ndim(o) - 1)), nv, o)
                 for nv, o in zip(new, old))


def single_colour_table(bits: int):
    """[256, 2] code pairs (a, b) of `bits`-bit endpoints: for value v, the pair whose four-colour 2/3
    point (2 E(a) + E(b) + 1) // 3 is nearest to v; ties to the smallest a, then the smallest b (step 8
    of REF-BC1)."""
    n = 1 << bits
    e = expand5(np.arange(n)) if bits == 5 else expand6(np.arange(n))
    pts = (2 * e[:, None] + e[None, :] + 1) // 3                 # [a, b]
    table = np.zeros((256, 2), dtype=np.int64)
    for v in range(256):
        k = int(np.argmin(np.abs(pts - v)))                      # first in (a, b) order
        table[v] = (k // n, k % n)
    return table


_SINGLE5 = None
_SINGLE6 = None


def bc1_encode_ref(blocks, return_sse: bool = False):
    """REF-BC1 on texel blocks uint8 [nb, 16, 3] -> BC1 words uint64 [nb] (and block SSE)."""
    p = np.asarray(blocks, dtype=np.int64)
    nb = p.shape[0]
    ar = np.arange(nb)
    # candidate A: farthest pair, lexicographically first on ties
    ii, jj = np.triu_indices(16, 1)
    d2 = ((p[:, ii, :] - p[:, jj, :]) ** 2).sum(axis=-1)       # [nb, 120]
    k = np.argmax(d2, axis=1)
    a0, a1 = p[ar, ii[k]], p[ar, jj[k]]
    # candidate B: inset bounding box with covariance-signed diagonal
    mn, mx = p.min(axis=1), p.max(axis=1)
    inset = (mx - mn) >> 4
    lo, hi = mn + inset, mx - inset
    m = np.argmax(mx - mn, axis=1)
    pm = p[ar, :, m]                                             # [nb, 16]
    cov = 16 * (p * pm[:, :, None]).sum(axis=1) - p.sum(axis=1) * pm.sum(axis=1)[:, None]
    flip = cov < 0
    b0 = np.where(flip, lo, hi)
    b1 = np.where(flip, hi, lo)
    st = _bc1_finish(quant565(a0), quant565(a1), p)
    st_b = _bc1_finish(quant565(b0), quant565(b1), p)
    st = _select(st_b[4] < st[4], st_b, st)
    for _ in range(2):
        ok, qa, qb = _bc1_refine(st[3], p)
        new = _bc1_finish(qa, qb, p)
        st = _select(ok & (new[4] < st[4]), new, st)
    # step 8: single-colour blocks
    global _SINGLE5, _SINGLE6
    if _SINGLE5 is None:
        _SINGLE5, _SINGLE6 = single_colour_table(5), single_colour_table(6)
    uniform = (p == p[:, :1, :]).all(axis=(1, 2))
    if uniform.any():
        v = p[:, 0, :]
        q0 = np.stack([_SINGLE5[v[:, 0], 0], _SINGLE6[v[:, 1], 0], _SINGLE5[v[:, 2], 0]], axis=-1)
        q1 = np.stack([_SINGLE5[v[:, 0], 1], _SINGLE6[v[:, 1], 1], _SINGLE5[v[:, 2], 1]], axis=-1)
        new = _bc1_finish(q0, q1, p)
        st = _select(uniform & (new[4] < st[4]), new, st)
    words = bc1_pack(st[0], st[1], st[2])
    return (words, st[4]) if return_sse else words


# ------------------------------------------------------------------------------------------------
# REF-BC4
# ------------------------------------------------------------------------------------------------
def _bc4_finish(e0, e1, v):
    """Codes by least squared error for endpoints e0, e1 [nb] and values v [nb, 16]."""
    pal = bc4_palette(e0, e1)                                    # [nb, 8 codes]
    order = bc4_logical_order(e0, e1)                            # [nb, 8]
    lpal = np.take_along_axis(pal, order, axis=1)                # by logical n
    err = (lpal[:, None, :] - v[:, :, None]) ** 2                # [nb, 16, 8]
    n = np.argmin(err, axis=2)
    codes = np.take_along_axis(order, n, axis=1)
    sse = np.take_along_axis(err, n[:, :, None], axis=2)[:, :, 0].sum(axis=1)
    return e0, e1, codes, n, sse


def _bc4_refine(e0, e1, n, v):
    eight = (e0 > e1)[:, None]
    inc = eight | ((n >= 1) & (n <= 6))
    a = np.where(eight, 7 - n, 6 - n) * inc
    b = np.where(eight, n, n - 1) * inc
    scale = np.where(e0 > e1, 7, 5)
    saa = (a * a).sum(axis=1)
    sbb = (b * b).sum(axis=1)
    sab = (a * b).sum(axis=1)
    sav = (a * v).sum(axis=1)
    sbv = (b * v).sum(axis=1)
    det = saa * sbb - sab * sab
    ok = det > 0
    d = np.where(ok, det, 1)
    num_a = np.clip(scale * (sbb * sav - sab * sbv), 0, 255 * d)
    num_b = np.clip(scale * (saa * sbv - sab * sav), 0, 255 * d)
    na = (2 * num_a + d) // (2 * d)
    nb_ = (2 * num_b + d) // (2 * d)
    keeps_mode = np.where(e0 > e1, na > nb_, na <= nb_)
    return ok & keeps_mode, na, nb_


def _bc4_refined(e0, e1, v):
    st = _bc4_finish(e0, e1, v)
    for _ in range(2):
        ok, na, nb_ = _bc4_refine(st[0], st[1], st[3], v)
        new = _bc4_finish(na, nb_, v)
        st = _select(ok & (new[4] < st[4]), new, st)
    return st


def bc4_encode_ref(blocks, return_sse: bool = False):
    """REF-BC4 on value blocks uint8 [nb, 16] (or [nb, 16, 1]) -> BC4 words uint64 [nb]."""
    v = np.asarray(blocks, dtype=np.int64)
    if v.ndim == 3:
        v = v[..., 0]
    st8 = _bc4_refined(v.max(axis=1), v.min(axis=1), v)
    interior = (v > 0) & (v < 255)
    has = interior.any(axis=1)
    lo = np.where(interior, v, 256).min(axis=1)
    hi = np.where(interior, v, -1).max(axis=1)
    st6 = _bc4_refined(np.where(has, lo, 0), np.where(has, hi, 0), v)
    st = _select(st6[4] < st8[4], st6, st8)
    words = bc4_pack(st[0], st[1], st[2])
    return (words, st[4]) if return_sse else words


def block_sse(words, blocks, fmt):
    """Integer SSE of decoded words [nb] against texel blocks [nb, 16, C]."""
    blocks = np.asarray(blocks, dtype=np.int64)
    if fmt == 1:
        dec = bc1_decode(words).astype(np.int64)
    else:
        dec = bc4_decode(words).astype(np.int64)[..., None]
        if blocks.ndim == 2:
            blocks = blocks[..., None]
    return ((dec - blocks) ** 2).sum(axis=(1, 2))
