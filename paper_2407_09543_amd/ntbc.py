"""ctypes binding of libntbc (argument marshalling only; every step runs in the HIP library).

Tensors are PyTorch CUDA (HIP) tensors; they provide device memory and the current stream.  Block
words are stored in int64 tensors (bit patterns of the uint64 little-endian BC words).  If the shared
library is not built, every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libntbc.so")

OK, EINVAL, EUNSUPPORTED, EHIP, ENONFINITE, ENOWORKSPACE = 0, -1, -2, -3, -4, -5
BC1, BC4 = 1, 4
FP32, BF16, FP8_E4M3, FP16 = 0, 1, 2, 3
GRID_F32, GRID_U8 = 0, 1
MAX_TEXTURES = 8
NTBC, NAIVE = 0, 1  # model variants: NTBC (Sec. 3.2) and the naive approach (Sec. 3.1)
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp16": FP16, "fp8": FP8_E4M3}


class NtbcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libntbc status {status}: {msg}")
        self.status = status


class ModelDesc(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("base_res", ctypes.c_int32),
                ("n_features", ctypes.c_int32), ("grid_dtype", ctypes.c_int32),
                ("hidden_width", ctypes.c_int32), ("n_hidden", ctypes.c_int32),
                ("n_textures", ctypes.c_int32), ("formats", ctypes.c_int32 * MAX_TEXTURES),
                ("blocks_w", ctypes.c_int32), ("blocks_h", ctypes.c_int32), ("variant", ctypes.c_int32)]


class FaithfulDesc(ctypes.Structure):
    _fields_ = [("ep_levels", ctypes.c_int32), ("ep_base_res", ctypes.c_int32), ("col_levels", ctypes.c_int32),
                ("col_base_res", ctypes.c_int32), ("grid_dtype", ctypes.c_int32), ("n_textures", ctypes.c_int32),
                ("formats", ctypes.c_int32 * MAX_TEXTURES), ("blocks_w", ctypes.c_int32), ("blocks_h", ctypes.c_int32)]


class FaithfulParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("ep_grid", "ep_scale", "ep_zero", "col_grid", "col_scale", "col_zero",
                                                 "ep_weights", "col_weights")]


class Params(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_void_p), ("grid_scale", ctypes.c_void_p),
                ("grid_zero", ctypes.c_void_p), ("weights", ctypes.c_void_p),
                ("fp8_scales", ctypes.c_void_p), ("flags", ctypes.c_int32)]

REUSE_PACKED = 1


class TrainStateC(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("grid", "weights", "m_grid", "v_grid", "m_weights",
                                                 "v_weights", "d_grid", "d_weights")]


class FaithfulTrainStateC(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in (
        "ep_grid", "col_grid", "ep_weights", "col_weights", "m_ep_grid", "v_ep_grid", "m_col_grid", "v_col_grid",
        "m_ep_weights", "v_ep_weights", "m_col_weights", "v_col_weights", "d_ep_grid", "d_col_grid", "d_ep_weights",
        "d_col_weights")]


class TargetsC(ctypes.Structure):
    _fields_ = [("ref_blocks", ctypes.c_void_p), ("texels", ctypes.c_void_p * MAX_TEXTURES),
                ("block_texels", ctypes.c_void_p * MAX_TEXTURES)]


class HParams(ctypes.Structure):
    _fields_ = [("lr_grid", ctypes.c_float), ("lr_mlp", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("temperature", ctypes.c_float),
                ("warmup", ctypes.c_int32), ("total_steps", ctypes.c_int32), ("qat", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("loss_weights", ctypes.c_float * 4),
                ("deterministic", ctypes.c_int32), ("stage2_from", ctypes.c_int32)]


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_F = ctypes.c_float

_SIGNATURES = {
    "ntbc_last_error": ([], ctypes.c_char_p),
    "ntbc_model_sizes": ([ctypes.POINTER(ModelDesc), ctypes.POINTER(_I64), ctypes.POINTER(_I32),
                          ctypes.POINTER(_I64)], ctypes.c_int),
    "ntbc_workspace_size": ([ctypes.POINTER(ModelDesc), _I32, _I64, ctypes.POINTER(_SZ)], ctypes.c_int),
    "ntbc_bc_encode_ref": ([_P, _I32, _I32, _I32, _I32, _P, _P, _P], ctypes.c_int),
    "ntbc_texels_to_blocks": ([_P, _I32, _I32, _I32, _I32, _P, _P], ctypes.c_int),
    "ntbc_bc_decode": ([_P, _I32, _I32, _I32, _P, _I32, _P], ctypes.c_int),
    "ntbc_block_sse": ([_P, _P, _I32, _I32, _I32, _I32, _P, _P], ctypes.c_int),
    "ntbc_fallback": ([_P, _P, _P, _P, _I64, _F, _F, _P, _P, _P], ctypes.c_int),
    "ntbc_fp8_calibrate": ([ctypes.POINTER(ModelDesc), ctypes.POINTER(Params), _I64, _P, _P, _SZ, _P], _I32),
    "ntbc_batch_table_size": ([_I32, ctypes.POINTER(_SZ)], _I32),
    "ntbc_batch_plan": ([ctypes.c_void_p, _I32, _I32, _P, _P, _SZ, ctypes.POINTER(_SZ)], _I32),
    "ntbc_batch_pack": ([_P, _P, _SZ, _P], _I32),
    "ntbc_infer_batch": ([_P, _P, _P, _SZ, _P, _P], _I32),
    "ntbc_batch_groups": ([_P, _P, _I32, ctypes.POINTER(_I32)], _I32),
    "ntbc_batch_set_waves": ([_P, _I32, _I32], _I32),
    "ntbc_infer_blocks": ([ctypes.POINTER(ModelDesc), ctypes.POINTER(Params), _I32, _I64, _I64, _P, _P,
                           _P, _SZ, _P], ctypes.c_int),
    "ntbc_infer_blocks_noalloc": ([ctypes.POINTER(ModelDesc), ctypes.POINTER(Params), _I32, _I64, _I64, _P, _P,
                                   _P], ctypes.c_int),
    "ntbc_forward": ([ctypes.POINTER(ModelDesc), _P, _P, _I32, _I32, _P, _I32, _P, _P, _SZ, _P], ctypes.c_int),
    "ntbc_backward": ([ctypes.POINTER(ModelDesc), _P, _P, _I32, _I32, _P, _I32, _P, _P, _P, _P, _SZ, _P],
                      ctypes.c_int),
    "ntbc_loss_grad": ([ctypes.POINTER(ModelDesc), ctypes.POINTER(TargetsC), _P, _P, _I32, _F, _P, _P, _P, _P],
                       ctypes.c_int),
    "ntbc_naive_loss_grad": ([ctypes.POINTER(ModelDesc), ctypes.POINTER(TargetsC), _P, _P, _I32, _I32, _P, _P, _P],
                             ctypes.c_int),
    "ntbc_faithful_sizes": ([ctypes.POINTER(FaithfulDesc), ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                             ctypes.POINTER(_SZ)], ctypes.c_int),
    "ntbc_faithful_infer": ([ctypes.POINTER(FaithfulDesc), ctypes.POINTER(FaithfulParams), _I64, _I64, _P, _P, _P, _SZ,
                             _P], ctypes.c_int),
    "ntbc_train_step": ([ctypes.POINTER(ModelDesc), ctypes.POINTER(TrainStateC), ctypes.POINTER(TargetsC), _P,
                         _I32, _I64, ctypes.POINTER(HParams), _P, _P, _SZ, _P], ctypes.c_int),
    "ntbc_faithful_train_size": ([ctypes.POINTER(FaithfulDesc), _I32, ctypes.POINTER(_SZ)], ctypes.c_int),
    "ntbc_faithful_train_step": ([ctypes.POINTER(FaithfulDesc), ctypes.POINTER(FaithfulTrainStateC),
                                  ctypes.POINTER(TargetsC), _P, _I32, _I64, ctypes.POINTER(HParams), _P, _P, _SZ, _P],
                                 ctypes.c_int),
    "ntbc_quantize_grid": ([ctypes.POINTER(ModelDesc), _P, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
    "ntbc_train_status": ([_P, _P], ctypes.c_int),
    "ntbc_batch_ids": ([ctypes.c_uint64, _I64, _I32, _I64, _P, _P], ctypes.c_int),
}


def lib():
    """Loads libntbc.so (built in-tree by paper_2407_09543_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2407_09543_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(handle, name, None)
            if fn is None:
                continue
            fn.argtypes = args
            fn.restype = res
        _lib = handle
    return _lib


def _check(status: int):
    if status != OK:
        raise NtbcError(status, lib().ntbc_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libntbc takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libntbc takes contiguous tensors")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_desc(n_levels, base_res, n_features, grid_u8, hidden, n_hidden, formats: Sequence[int],
              blocks_w, blocks_h, variant: int = 0) -> ModelDesc:
    d = ModelDesc()
    d.n_levels, d.base_res, d.n_features = n_levels, base_res, n_features
    d.grid_dtype = GRID_U8 if grid_u8 else GRID_F32
    d.hidden_width, d.n_hidden = hidden, n_hidden
    d.n_textures = len(formats)
    for i, f in enumerate(formats):
        d.formats[i] = int(f)
    d.blocks_w, d.blocks_h = blocks_w, blocks_h
    d.variant = int(variant)
    return d


def desc_from_config(cfg) -> ModelDesc:
    """ModelDesc of a config object with the fields of synth.ModelConfig."""
    return make_desc(cfg.n_levels, cfg.base_res, cfg.n_features, cfg.grid_u8, cfg.hidden, cfg.n_hidden,
                     cfg.formats, cfg.blocks_w, cfg.blocks_h, NAIVE if getattr(cfg, "variant", "ntbc") == "naive" else NTBC)


def model_sizes(desc: ModelDesc):
    nw, hd, gv = _I64(), _I32(), _I64()
    _check(lib().ntbc_model_sizes(ctypes.byref(desc), ctypes.byref(nw), ctypes.byref(hd), ctypes.byref(gv)))
    return nw.value, hd.value, gv.value


def workspace_size(desc: ModelDesc, precision: int, batch: int = 0) -> int:
    out = _SZ()
    _check(lib().ntbc_workspace_size(ctypes.byref(desc), precision, batch, ctypes.byref(out)))
    return out.value


# ---------------------------------------------------------------------------------------------- BC
def _tex_dims(texels: torch.Tensor, fmt: int):
    ch = 3 if fmt == BC1 else 1
    if fmt == BC1 and (texels.dim() != 3 or texels.shape[2] != 3):
        raise ValueError("BC1 textures are [H, W, 3] uint8")
    if fmt == BC4 and texels.dim() not in (2, 3):
        raise ValueError("BC4 textures are [H, W] uint8")
    if texels.dtype != torch.uint8:
        raise ValueError("textures are uint8")
    h, w = texels.shape[0], texels.shape[1]
    return w, h, w * ch


def encode_ref(texels: torch.Tensor, fmt: int, return_sse: bool = False):
    """Reference BC encoding of a device texture -> int64 tensor of BC words [H/4 * W/4]."""
    w, h, pitch = _tex_dims(texels, fmt)
    out = torch.empty((h // 4) * (w // 4), dtype=torch.int64, device=texels.device)
    sse = torch.empty(out.shape, dtype=torch.int32, device=texels.device) if return_sse else None
    _check(lib().ntbc_bc_encode_ref(_ptr(texels), w, h, pitch, fmt, _ptr(out), _ptr(sse), _stream()))
    return (out, sse) if return_sse else out


def decode(blocks: torch.Tensor, width: int, height: int, fmt: int) -> torch.Tensor:
    ch = 3 if fmt == BC1 else 1
    shape = (height, width, 3) if fmt == BC1 else (height, width)
    out = torch.empty(shape, dtype=torch.uint8, device=blocks.device)
    _check(lib().ntbc_bc_decode(_ptr(blocks), width, height, fmt, _ptr(out), width * ch, _stream()))
    return out


def block_sse(blocks: torch.Tensor, texels: torch.Tensor, fmt: int) -> torch.Tensor:
    w, h, pitch = _tex_dims(texels, fmt)
    out = torch.empty(blocks.shape, dtype=torch.int32, device=blocks.device)
    _check(lib().ntbc_block_sse(_ptr(blocks), _ptr(texels), w, h, pitch, fmt, _ptr(out), _stream()))
    return out


def fallback(ntbc_words, ref_words, sse_ntbc, sse_ref, kappa: float, delta: float):
    """Per-block judge: (words, replaced count as a device int32 tensor)."""
    out = torch.empty_like(ntbc_words)
    count = torch.zeros(1, dtype=torch.int32, device=ntbc_words.device)
    _check(lib().ntbc_fallback(_ptr(ntbc_words), _ptr(ref_words), _ptr(sse_ntbc), _ptr(sse_ref),
                               ntbc_words.numel(), kappa, delta, _ptr(out), _ptr(count), _stream()))
    return out, count


# -------------------------------------------------------------------------------------- inference
class Model:
    """Device-resident inference parameters of one material (the caller keeps the tensors alive)."""

    def __init__(self, desc: ModelDesc, weights: torch.Tensor, grid: torch.Tensor,
                 grid_scale: Optional[torch.Tensor] = None, grid_zero: Optional[torch.Tensor] = None,
                 fp8_scales: Optional[torch.Tensor] = None):
        self.desc = desc
        self.weights = weights.contiguous()
        self.grid = grid.contiguous()
        self.grid_scale = grid_scale
        self.grid_zero = grid_zero
        self.fp8_scales = fp8_scales
        self.n_weights, self.head_dim, self.grid_vertices = model_sizes(desc)
        self._ws = {}

    def params(self) -> Params:
        p = Params()
        p.grid = self.grid.data_ptr()
        p.grid_scale = self.grid_scale.data_ptr() if self.grid_scale is not None else None
        p.grid_zero = self.grid_zero.data_ptr() if self.grid_zero is not None else None
        p.weights = self.weights.data_ptr()
        p.fp8_scales = self.fp8_scales.data_ptr() if self.fp8_scales is not None else None
        return p

    def workspace(self, precision: int) -> torch.Tensor:
        if precision not in self._ws:
            n = workspace_size(self.desc, precision, 0)
            self._ws[precision] = torch.empty(max(n, 1), dtype=torch.uint8, device=self.weights.device)
        return self._ws[precision]

    def fp8_calibrate(self, n_sample: int = 65536) -> torch.Tensor:
        """Per-layer FP8 scales [n_layers][2] = (s_x, s_w) from ntbc_fp8_calibrate; kept on the model for
        FP8 inference."""
        n_layers = len(self._layer_count())
        scales = torch.empty((n_layers, 2), dtype=torch.float32, device=self.weights.device)
        ws = self.workspace(FP8_E4M3)
        _check(lib().ntbc_fp8_calibrate(ctypes.byref(self.desc), ctypes.byref(self.params()), n_sample, _ptr(scales),
                                        _ptr(ws), ws.numel(), _stream()))
        self.fp8_scales = scales
        return scales

    def _layer_count(self):
        return range(self.desc.n_hidden + 1)

    def infer(self, precision: int = BF16, first_block: int = 0, n_blocks: Optional[int] = None,
              heads: bool = False, out: Optional[torch.Tensor] = None, reuse_packed: bool = False):
        """Packed blocks int64 [n_textures, n_blocks] (and heads float32 [n_blocks, head_dim]).

        reuse_packed: skip re-packing the weights (valid only after an earlier call at the same
        precision with unchanged weights)."""
        if n_blocks is None:
            n_blocks = self.desc.blocks_w * self.desc.blocks_h - first_block
        dev = self.weights.device
        if out is None:
            out = torch.empty((self.desc.n_textures, n_blocks), dtype=torch.int64, device=dev)
        h = torch.empty((n_blocks, self.head_dim), dtype=torch.float32, device=dev) if heads else None
        ws = self.workspace(precision)
        p = self.params()
        p.flags = REUSE_PACKED if reuse_packed else 0
        _check(lib().ntbc_infer_blocks(ctypes.byref(self.desc), ctypes.byref(p), precision, first_block,
                                       n_blocks, _ptr(out), _ptr(h), _ptr(ws), ws.numel(), _stream()))
        return (out, h) if heads else out

    def infer_noalloc(self, precision: int = BF16, first_block: int = 0, n_blocks: Optional[int] = None,
                      heads: bool = False, out: Optional[torch.Tensor] = None, reuse_packed: bool = False):
        """As infer(), through ntbc_infer_blocks_noalloc: the library's static per-device scratch holds the
        packed weights, so the call allocates nothing on the device (pass `out` to allocate nothing here
        either)."""
        if n_blocks is None:
            n_blocks = self.desc.blocks_w * self.desc.blocks_h - first_block
        dev = self.weights.device
        if out is None:
            out = torch.empty((self.desc.n_textures, n_blocks), dtype=torch.int64, device=dev)
        h = torch.empty((n_blocks, self.head_dim), dtype=torch.float32, device=dev) if heads else None
        p = self.params()
        p.flags = REUSE_PACKED if reuse_packed else 0
        _check(lib().ntbc_infer_blocks_noalloc(ctypes.byref(self.desc), ctypes.byref(p), precision, first_block,
                                               n_blocks, _ptr(out), _ptr(h), _stream()))
        return (out, h) if heads else out


class FaithfulModel:
    """One model of the paper's own layout (endpoint network + per-texel colour network, SELU, half
    precision; ntbc_faithful_infer).  Grids are device tensors of 2 features per vertex (uint8 with
    per-level scale/zero, or float32); weights are the canonical FP32 layouts of the two networks."""

    def __init__(self, formats, blocks_w: int, blocks_h: int, ep_grid, col_grid, ep_weights, col_weights,
                 ep_levels: int = 7, ep_base_res: int = 16, col_levels: int = 8, col_base_res: int = 16,
                 ep_scale=None, ep_zero=None, col_scale=None, col_zero=None):
        d = FaithfulDesc()
        d.ep_levels, d.ep_base_res, d.col_levels, d.col_base_res = ep_levels, ep_base_res, col_levels, col_base_res
        d.grid_dtype = GRID_U8 if ep_grid.dtype == torch.uint8 else GRID_F32
        d.n_textures = len(formats)
        for i, f in enumerate(formats):
            d.formats[i] = int(f)
        d.blocks_w, d.blocks_h = blocks_w, blocks_h
        self.desc = d
        self.tensors = [t.contiguous() if t is not None else None
                        for t in (ep_grid, ep_scale, ep_zero, col_grid, col_scale, col_zero, ep_weights, col_weights)]
        self.params = FaithfulParams(*[t.data_ptr() if t is not None else None for t in self.tensors])
        ne, nc, ws = _I64(), _I64(), _SZ()
        _check(lib().ntbc_faithful_sizes(ctypes.byref(d), ctypes.byref(ne), ctypes.byref(nc), ctypes.byref(ws)))
        self.n_ep_weights, self.n_col_weights = ne.value, nc.value
        self.ws = torch.empty(max(ws.value, 1), dtype=torch.uint8, device=ep_grid.device)
        e = sum(6 if f == BC1 else 2 for f in formats)
        c = sum(3 if f == BC1 else 1 for f in formats)
        self.head_dim = e + 16 * c

    def infer(self, first_block: int = 0, n_blocks: Optional[int] = None, heads: bool = False,
              out: Optional[torch.Tensor] = None):
        """Packed blocks int64 [n_textures, n_blocks] (and heads float32 [n_blocks, E + 16 C])."""
        if n_blocks is None:
            n_blocks = self.desc.blocks_w * self.desc.blocks_h - first_block
        dev = self.ws.device
        if out is None:
            out = torch.empty((self.desc.n_textures, n_blocks), dtype=torch.int64, device=dev)
        h = torch.empty((n_blocks, self.head_dim), dtype=torch.float32, device=dev) if heads else None
        _check(lib().ntbc_faithful_infer(ctypes.byref(self.desc), ctypes.byref(self.params), first_block, n_blocks,
                                         _ptr(out), _ptr(h), _ptr(self.ws), self.ws.numel(), _stream()))
        return (out, h) if heads else out


class BatchItemC(ctypes.Structure):
    _fields_ = [("desc", ModelDesc), ("params", Params), ("first_block", ctypes.c_int64),
                ("n_blocks", ctypes.c_int64), ("blocks_out", ctypes.c_void_p), ("model_id", ctypes.c_int32)]


def mip_desc(desc: ModelDesc, level: int) -> ModelDesc:
    """The block grid of mip `level` of a model (the network queried at that mip's block centres)."""
    d = ModelDesc.from_buffer_copy(desc)
    d.blocks_w = max(1, desc.blocks_w >> level)
    d.blocks_h = max(1, desc.blocks_h >> level)
    return d


class Batch:
    """A planned batched decode: items (model, desc, first_block, n_blocks) -> one output tensor per
    item; run() issues one launch per kernel instance (capturable in a HIP graph)."""

    def __init__(self, entries, precision: int = BF16, tiles=None):
        """tiles: {instance key: waves} tile shapes (autotune.key); None = the committed autotuner table,
        {} = the default shape everywhere."""
        self.models = [e[0] for e in entries]
        n = len(entries)
        dev = self.models[0].weights.device
        self.outputs = []
        arr = (BatchItemC * n)()
        ids = {}
        for i, (model, desc, first, count) in enumerate(entries):
            out = torch.empty((desc.n_textures, count), dtype=torch.int64, device=dev)
            self.outputs.append(out)
            arr[i].desc = desc
            arr[i].params = model.params()
            arr[i].first_block = first
            arr[i].n_blocks = count
            arr[i].blocks_out = out.data_ptr()
            arr[i].model_id = ids.setdefault(id(model), len(ids))
        self._arr = arr
        tb = _SZ()
        _check(lib().ntbc_batch_table_size(n, ctypes.byref(tb)))
        self.table = (ctypes.c_uint8 * tb.value)()
        wsb = _SZ()
        _check(lib().ntbc_batch_plan(ctypes.addressof(arr), n, precision, None, ctypes.addressof(self.table), tb.value,
                                     ctypes.byref(wsb)))
        self.ws = torch.empty(max(wsb.value, 256), dtype=torch.uint8, device=dev)
        _check(lib().ntbc_batch_plan(ctypes.addressof(arr), n, precision, self.ws.data_ptr(),
                                     ctypes.addressof(self.table), tb.value, ctypes.byref(wsb)))
        self.table_dev = torch.frombuffer(bytearray(bytes(self.table)), dtype=torch.uint8).to(dev)
        self.n = n
        from . import autotune
        autotune.apply(self, autotune.load_table() if tiles is None else tiles)
        _check(lib().ntbc_batch_pack(ctypes.addressof(self.table), _ptr(self.ws), self.ws.numel(), _stream()))

    def groups(self):
        """Kernel instances of the plan: dicts of precision, hidden, ks0, nh, nb1, nb4, waves, items."""
        n = _I32()
        _check(lib().ntbc_batch_groups(ctypes.addressof(self.table), None, 0, ctypes.byref(n)))
        buf = (_I32 * (8 * max(n.value, 1)))()
        _check(lib().ntbc_batch_groups(ctypes.addressof(self.table), buf, n.value, ctypes.byref(n)))
        keys = ("precision", "hidden", "ks0", "nh", "nb1", "nb4", "waves", "items")
        return [dict(zip(keys, buf[8 * g:8 * g + 8])) for g in range(n.value)]

    def set_waves(self, group: int, waves: int):
        """Tile shape (waves of 32 positions per workgroup) of one kernel instance; the device copy of
        the plan is refreshed."""
        _check(lib().ntbc_batch_set_waves(ctypes.addressof(self.table), group, waves))
        self.table_dev.copy_(torch.frombuffer(bytearray(bytes(self.table)), dtype=torch.uint8))

    def run(self, stamps: Optional[torch.Tensor] = None):
        """Decodes every item into self.outputs; stamps (uint64 as int64 [n + 1]) receive the start and
        per-item completion times of the 100 MHz real-time counter."""
        _check(lib().ntbc_infer_batch(ctypes.addressof(self.table), _ptr(self.table_dev), _ptr(self.ws), self.ws.numel(),
                                      _ptr(stamps), _stream()))
        return self.outputs


# -------------------------------------------------------------------------------------- training
def _scratch(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def forward(desc: ModelDesc, grid: torch.Tensor, weights: torch.Tensor, ids: torch.Tensor, qat: bool = False,
            precision: int = FP32) -> torch.Tensor:
    """Sigmoid heads [n, head_dim] of block positions ids (int32) from the FP32 master parameters."""
    n = ids.numel()
    _, head_dim, _ = model_sizes(desc)
    out = torch.empty((n, head_dim), dtype=torch.float32, device=grid.device)
    ws = _scratch(workspace_size(desc, precision, max(n, 1)), grid.device)
    _check(lib().ntbc_forward(ctypes.byref(desc), _ptr(grid), _ptr(weights), int(qat), precision, _ptr(ids), n,
                              _ptr(out), _ptr(ws), ws.numel(), _stream()))
    return out


def backward(desc: ModelDesc, grid, weights, ids, d_heads, qat: bool = False, precision: int = FP32):
    """(d_grid, d_weights) of sum(d_heads * heads); the forward activations are recomputed."""
    n = ids.numel()
    dg = torch.zeros_like(grid)
    dw = torch.zeros_like(weights)
    ws = _scratch(workspace_size(desc, precision, max(n, 1)), grid.device)
    _check(lib().ntbc_backward(ctypes.byref(desc), _ptr(grid), _ptr(weights), int(qat), precision, _ptr(ids), n,
                               _ptr(d_heads.contiguous()), _ptr(dg), _ptr(dw), _ptr(ws), ws.numel(), _stream()))
    return dg, dw


class NTBCFunction(torch.autograd.Function):
    """Heads [n, head_dim] as a differentiable function of the FP32 grid and MLP weights.  The
    backward calls ntbc_backward, which recomputes the forward activations instead of keeping them
    (Sec. 3.2; the grid gradient is a scatter-add through the bilinear weights, Sec. 3.3 with QAT)."""

    @staticmethod
    def forward(ctx, grid, weights, ids, desc, qat=False):
        ctx.desc, ctx.qat = desc, bool(qat)
        ctx.save_for_backward(grid, weights, ids)
        return forward(desc, grid, weights, ids, qat)

    @staticmethod
    def backward(ctx, d_heads):
        grid, weights, ids = ctx.saved_tensors
        dg, dw = backward(ctx.desc, grid, weights, ids, d_heads, ctx.qat)
        return dg, dw, None, None, None


def texels_to_blocks(texels: torch.Tensor, fmt: int) -> torch.Tensor:
    """Block-major copy of a device texture: uint8 [n_blocks, 16, channels] (ntbc_texels_to_blocks)."""
    w, h, pitch = _tex_dims(texels, fmt)
    ch = 3 if fmt == BC1 else 1
    out = torch.empty(((h // 4) * (w // 4), 16, ch), dtype=torch.uint8, device=texels.device)
    _check(lib().ntbc_texels_to_blocks(_ptr(texels), w, h, pitch, fmt, _ptr(out), _stream()))
    return out


class Targets:
    """Reference blocks [n_textures, n_positions] (int64) and the textures (uint8, device; [H, W, 3] for
    BC1, [H, W] for BC4).  block_major: also keep block-major copies, which the losses then read."""

    def __init__(self, ref_blocks: torch.Tensor, textures: Sequence[torch.Tensor], block_major: bool = True):
        self.ref_blocks = ref_blocks.contiguous()
        self.textures = [t.contiguous() for t in textures]
        self.c = TargetsC()
        self.c.ref_blocks = self.ref_blocks.data_ptr()
        self.blocks = []
        for i, t in enumerate(self.textures):
            self.c.texels[i] = t.data_ptr()
            if block_major:
                self.blocks.append(texels_to_blocks(t, BC1 if t.dim() == 3 and t.shape[2] == 3 else BC4))
                self.c.block_texels[i] = self.blocks[-1].data_ptr()


def loss_grad(desc: ModelDesc, targets: Targets, heads: torch.Tensor, ids: torch.Tensor,
              temperature: float = 0.01, loss_weights=(1.0, 1.0, 1.0, 1.0)):
    """(losses float32[5] = L_e, L_c, L_cd_e, L_cd_c, nonfinite flag; dL/dheads)."""
    losses = torch.empty(5, dtype=torch.float32, device=heads.device)
    dh = torch.empty_like(heads)
    lw = torch.tensor(loss_weights, dtype=torch.float32, device=heads.device)
    _check(lib().ntbc_loss_grad(ctypes.byref(desc), ctypes.byref(targets.c), _ptr(heads.contiguous()), _ptr(ids),
                                ids.numel(), temperature, _ptr(lw), _ptr(losses), _ptr(dh), _stream()))
    return losses, dh


def naive_loss_grad(desc: ModelDesc, targets: Targets, heads: torch.Tensor, ids: torch.Tensor, stage: int):
    """Naive-approach loss (losses float32[5] = L, 0, 0, 0, nonfinite flag; dL/dheads) of stage 1 or 2."""
    losses = torch.empty(5, dtype=torch.float32, device=heads.device)
    dh = torch.empty_like(heads)
    _check(lib().ntbc_naive_loss_grad(ctypes.byref(desc), ctypes.byref(targets.c), _ptr(heads.contiguous()),
                                      _ptr(ids), ids.numel(), stage, _ptr(losses), _ptr(dh), _stream()))
    return losses, dh


def quantize_grid(desc: ModelDesc, grid: torch.Tensor):
    """(codes uint8 [V, F], scale float32 [L], zero int32 [L]) of an FP32 grid."""
    codes = torch.empty(grid.shape, dtype=torch.uint8, device=grid.device)
    scale = torch.empty(desc.n_levels, dtype=torch.float32, device=grid.device)
    zero = torch.empty(desc.n_levels, dtype=torch.int32, device=grid.device)
    ws = _scratch(1024, grid.device)
    _check(lib().ntbc_quantize_grid(ctypes.byref(desc), _ptr(grid), _ptr(codes), _ptr(scale), _ptr(zero), _ptr(ws),
                                    ws.numel(), _stream()))
    return codes, scale, zero


class Trainer:
    """FP32 master parameters, Adam state and scratch of one material on the device."""

    def __init__(self, desc: ModelDesc, grid: torch.Tensor, weights: torch.Tensor, targets: Targets, batch: int,
                 total_steps: int, lr_grid: float = 0.01, lr_mlp: float = 0.005, temperature: float = 0.01,
                 warmup: int = 10, loss_weights=(1.0, 1.0, 1.0, 1.0), precision: int = FP32,
                 deterministic: bool = False, stage2_from: Optional[int] = None):
        self.desc = desc
        self.grid = grid.clone().contiguous()
        self.weights = weights.clone().contiguous()
        self.targets = targets
        self.batch = batch
        dev = grid.device
        self.m_grid, self.v_grid = torch.zeros_like(self.grid), torch.zeros_like(self.grid)
        self.m_w, self.v_w = torch.zeros_like(self.weights), torch.zeros_like(self.weights)
        self.d_grid, self.d_w = torch.zeros_like(self.grid), torch.zeros_like(self.weights)
        self.ws = _scratch(workspace_size(desc, precision, batch), dev)
        self.losses = torch.zeros(5, dtype=torch.float32, device=dev)
        self.state = TrainStateC(*[t.data_ptr() for t in (self.grid, self.weights, self.m_grid, self.v_grid,
                                                          self.m_w, self.v_w, self.d_grid, self.d_w)])
        # naive variant: the paper's two stages split the steps 80/20 (Sec. 3.1)
        if stage2_from is None:
            stage2_from = (4 * total_steps) // 5
        self.h = HParams(lr_grid, lr_mlp, 0.9, 0.999, 1e-15, temperature, warmup, total_steps, 0, precision,
                         (ctypes.c_float * 4)(*loss_weights), int(deterministic), int(stage2_from))

    def step(self, ids: torch.Tensor, step: int, qat: bool = False) -> torch.Tensor:
        """One step on the batch ids (int32, device); returns the device losses[5] (overwritten)."""
        self.h.qat = int(qat)
        _check(lib().ntbc_train_step(ctypes.byref(self.desc), ctypes.byref(self.state), ctypes.byref(self.targets.c),
                                     _ptr(ids), ids.numel(), step, ctypes.byref(self.h), _ptr(self.losses),
                                     _ptr(self.ws), self.ws.numel(), _stream()))
        return self.losses

    def status(self) -> int:
        """ntbc_train_status of the last step: OK, or ENONFINITE when it skipped its update (waits for
        the stream)."""
        return lib().ntbc_train_status(_ptr(self.losses), _stream())


class FaithfulTrainer:
    """FP32 master parameters, Adam state and scratch of one model of the paper's own layout
    (ntbc_faithful_train_step): grids [V][2] float32, canonical FP32 weights of each network."""

    def __init__(self, formats, blocks_w: int, blocks_h: int, ep_grid: torch.Tensor, col_grid: torch.Tensor,
                 ep_weights: torch.Tensor, col_weights: torch.Tensor, targets: Targets, batch: int, total_steps: int,
                 ep_levels: int = 7, ep_base_res: int = 16, col_levels: int = 8, col_base_res: int = 16,
                 lr_grid: float = 0.01, lr_mlp: float = 0.005, temperature: float = 0.01, warmup: int = 10,
                 loss_weights=(1.0, 1.0, 1.0, 1.0), deterministic: bool = False):
        d = FaithfulDesc()
        d.ep_levels, d.ep_base_res, d.col_levels, d.col_base_res = ep_levels, ep_base_res, col_levels, col_base_res
        d.grid_dtype = GRID_F32
        d.n_textures = len(formats)
        for i, f in enumerate(formats):
            d.formats[i] = int(f)
        d.blocks_w, d.blocks_h = blocks_w, blocks_h
        self.desc = d
        self.formats = list(formats)
        self.targets = targets
        self.params = [t.clone().contiguous() for t in (ep_grid, col_grid, ep_weights, col_weights)]
        self.ep_grid, self.col_grid, self.ep_weights, self.col_weights = self.params
        self.m = [torch.zeros_like(t) for t in self.params]
        self.v = [torch.zeros_like(t) for t in self.params]
        self.grads = [torch.zeros_like(t) for t in self.params]
        self.d_ep_grid, self.d_col_grid, self.d_ep_weights, self.d_col_weights = self.grads
        ptrs = self.params + [self.m[0], self.v[0], self.m[1], self.v[1], self.m[2], self.v[2], self.m[3], self.v[3]] + \
            self.grads
        self.state = FaithfulTrainStateC(*[t.data_ptr() for t in ptrs])
        ws = _SZ()
        _check(lib().ntbc_faithful_train_size(ctypes.byref(d), batch, ctypes.byref(ws)))
        self.ws = _scratch(ws.value, ep_grid.device)
        self.losses = torch.zeros(5, dtype=torch.float32, device=ep_grid.device)
        self.h = HParams(lr_grid, lr_mlp, 0.9, 0.999, 1e-15, temperature, warmup, total_steps, 0, FP32,
                         (ctypes.c_float * 4)(*loss_weights), int(deterministic), 0)

    def step(self, ids: torch.Tensor, step: int, qat: bool = False) -> torch.Tensor:
        """One step on the block batch ids (int32, device); returns the device losses[5] (overwritten)."""
        self.h.qat = int(qat)
        _check(lib().ntbc_faithful_train_step(ctypes.byref(self.desc), ctypes.byref(self.state),
                                              ctypes.byref(self.targets.c), _ptr(ids), ids.numel(), step,
                                              ctypes.byref(self.h), _ptr(self.losses), _ptr(self.ws), self.ws.numel(),
                                              _stream()))
        return self.losses


def batch_ids(seed: int, step: int, batch: int, n_positions: int, out: Optional[torch.Tensor] = None,
              device="cuda") -> torch.Tensor:
    """Device int32 batch of block ids (SplitMix64 stream keyed by seed and step)."""
    if out is None:
        out = torch.empty(batch, dtype=torch.int32, device=device)
    _check(lib().ntbc_batch_ids(seed, step, batch, n_positions, _ptr(out), _stream()))
    return out
