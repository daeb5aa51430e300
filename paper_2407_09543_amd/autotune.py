"""Tile-shape autotuner of the batched load-time decode.

A planned batch (ntbc.Batch) runs one launch per fused-kernel instance (precision, hidden width,
first-layer K-steps, unrolled middle layers, register-epilogue texture mix).  Each BF16 instance exists
with tiles of 2, 4 and 8 waves of 32 block positions per workgroup: fewer waves give more workgroups
and a smaller LDS footprint, more waves share each weight chunk over more positions.  tune() times the
whole batch with every instance at every shape (the other instances at their best so far, one pass in
plan order) and keeps the fastest; the result is a table keyed by the instance, which Batch applies
when it plans (`tiles=`; by default the committed table below).

    python -m paper_2407_09543_amd.autotune --write     # times the 16-material mip-chain workload on
                                                        # the GPU and writes batch_tiles.json
"""
from __future__ import annotations

import json
import os
import sys

import torch

from . import ntbc

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_tiles.json")
SHAPES = (2, 4, 8)


def key(g) -> str:
    """Table key of a kernel instance (a dict from Batch.groups())."""
    return f"{g['precision']}/{g['hidden']}/{g['ks0']}/{g['nh']}/{g['nb1']}/{g['nb4']}"


def _time(batch, reps: int, warmup: int = 2) -> float:
    """Milliseconds of one batch run (HIP events on the current stream), mean over `reps` runs."""
    for _ in range(warmup):
        batch.run()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        batch.run()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / reps


def tune(batch, reps: int = 10):
    """{key: {"waves": best, "ms": {shape: batch ms}}} for every instance of the batch (non-BF16
    instances have the 4-wave shape only); leaves the batch at the chosen shapes."""
    table = {}
    for gi, g in enumerate(batch.groups()):
        times = {}
        for w in SHAPES:
            try:
                batch.set_waves(gi, w)
            except ntbc.NtbcError:
                continue
            times[w] = _time(batch, reps)
        best = min(times, key=times.get)
        batch.set_waves(gi, best)
        table[key(g)] = {"waves": best, "ms": times}
    return table


def load_table(path: str = TABLE_PATH):
    """{key: waves} from a written table, {} if there is none."""
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        data = json.load(fh)
    return {k: int(v["waves"]) for k, v in data.get("instances", {}).items()}


def apply(batch, tiles) -> None:
    """Sets every instance of the batch that the table names to its shape."""
    for gi, g in enumerate(batch.groups()):
        w = tiles.get(key(g))
        if w is not None and w != g["waves"]:
            batch.set_waves(gi, w)


def batched_decode_workload(device="cuda:0"):
    """The batched load-time decode workload: 16 materials m = 0..15 of size 512 * 2^(m mod 4), MLP width
    64 (1 + m // 4), 3 + (m mod 3) textures (the first min(2, n - 1) BC1, the rest BC4), 8 grid levels
    from 8 with 8 uint8 features, random parameters of those shapes (seed 100 + m), each with its full
    mip chain (a mip is the network queried at the block centres of its own block grid).  Returns
    (batch entries, material of each entry, per material the models of its mips)."""
    import numpy as np
    from . import synth
    dev = torch.device(device)
    entries, mat_of, per_mat = [], [], []
    for m in range(16):
        size, width, nt = 512 << (m % 4), 64 * (1 + m // 4), 3 + (m % 3)
        n_bc1 = min(2, nt - 1)
        cfg = synth.ModelConfig(8, 8, 8, True, width, 3, tuple([synth.BC1] * n_bc1 + [synth.BC4] * (nt - n_bc1)),
                                size // 4, size // 4)
        layers = synth.init_weights(cfg, 100 + m)
        codes, _, _ = synth.random_u8_grid(cfg, 100 + m)
        model = ntbc.Model(ntbc.desc_from_config(cfg), torch.from_numpy(synth.flatten_weights(layers)).to(dev),
                           torch.from_numpy(codes).to(dev),
                           torch.from_numpy(np.full(cfg.n_levels, 0.7 / 128, np.float32)).to(dev),
                           torch.from_numpy(np.full(cfg.n_levels, 128, np.int32)).to(dev))
        mips = []
        level = 0
        while (cfg.blocks_w >> level) >= 1:
            d = ntbc.mip_desc(model.desc, level)
            entries.append((model, d, 0, d.blocks_w * d.blocks_h))
            mat_of.append(m)
            mips.append(ntbc.Model(d, model.weights, model.grid, model.grid_scale, model.grid_zero))
            level += 1
        per_mat.append(mips)
    return entries, mat_of, per_mat


def _main(argv):
    write = "--write" in argv
    entries, _, _ = batched_decode_workload()
    batch = ntbc.Batch(entries, ntbc.BF16, tiles={})
    table = tune(batch)
    out = {"workload": "16 materials 512^2..4096^2 with full mip chains, widths 64..256, 3-5 textures "
                       "(the batched load-time decode), BF16",
           "device": torch.cuda.get_device_name(0),
           "instances": {k: {"waves": v["waves"], "ms": {str(w): t for w, t in v["ms"].items()}}
                         for k, v in table.items()}}
    print(json.dumps(out, indent=1), flush=True)
    if write:
        with open(TABLE_PATH, "w") as fh:
            json.dump(out, fh, indent=1)
            fh.write("\n")


if __name__ == "__main__":
    _main(sys.argv[1:])
