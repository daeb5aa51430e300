"""Batched load-time decode: many materials and mip levels in one launch per kernel instance.

Every item's blocks equal ntbc_infer_blocks on the same model, block grid and range (the same fused
kernel and arithmetic), a sample of them equals the oracle of the same precision within the 16-bit
tolerances with every differing block a tie, the batch replays identically from a HIP graph, and the
completion stamps are ordered after the start stamp."""
import dataclasses

import numpy as np
import pytest
import torch

from cases import model_inputs, oracle_levels
from util import ensure_built, log, u64
from oracle import metrics as OM
from oracle import ntbc as ON
from paper_2407_09543_amd import ntbc, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    assert torch.cuda.is_available()


def _device_model(cfg, flat, g):
    desc = ntbc.desc_from_config(cfg)
    w = torch.from_numpy(flat).cuda()
    if "codes" in g:
        return ntbc.Model(desc, w, torch.from_numpy(g["codes"]).cuda(), torch.from_numpy(g["scale"]).cuda(),
                          torch.from_numpy(g["zero"]).cuda())
    return ntbc.Model(desc, w, torch.from_numpy(g["grid"]).cuda())


def _materials():
    """Five models of different widths / first-layer shapes / texture mixes, each with its mip chain as
    items.  In BF16 the paper-scale model (two BC1 + three BC4, width 256) and the two 64-input models
    (two BC1 + two BC4 at width 128, two BC1 + one BC4 at width 64, run-time layer count) use the
    register-resident BC epilogue in the batch, while their single launches use the LDS-staged one."""
    out = []
    w128 = dataclasses.replace(synth.config_mid(256), n_levels=8, base_res=2, hidden=128, n_hidden=2, formats=(1, 1, 4, 4))
    w64 = dataclasses.replace(synth.config_mid(128), n_levels=8, base_res=2, hidden=64, n_hidden=3, formats=(1, 1, 4))
    for cfg, seed in ((synth.config_small(256), 1), (synth.config_mid(512), 2), (synth.config_paper_scale(1024), 3),
                      (w128, 4), (w64, 5)):
        flat, layers, g = model_inputs(cfg, seed)
        out.append((cfg, layers, g, _device_model(cfg, flat, g)))
    return out


def _entries(mats):
    entries, meta = [], []
    for k, (cfg, layers, g, model) in enumerate(mats):
        level = 0
        while (cfg.blocks_w >> level) >= 1:
            d = ntbc.mip_desc(model.desc, level)
            n = d.blocks_w * d.blocks_h
            entries.append((model, d, 0, n))
            meta.append((k, level))
            level += 1
        # a partial range of the top level as well
        entries.append((model, model.desc, 37, model.desc.blocks_w * model.desc.blocks_h - 37 - 5))
        meta.append((k, -1))
    return entries, meta


@pytest.mark.parametrize("precision", [ntbc.BF16, ntbc.FP16])
def test_batch_equals_single_launches_and_oracle(precision):
    mats = _materials()
    entries, meta = _entries(mats)
    batch = ntbc.Batch(entries, precision)
    stamps = torch.zeros(len(entries) + 1, dtype=torch.int64, device="cuda")
    outs = batch.run(stamps)
    torch.cuda.synchronize()
    emu = {ntbc.BF16: "bf16", ntbc.FP16: "fp16"}[precision]
    tol = {ntbc.BF16: 1e-2, ntbc.FP16: 2e-3}[precision]
    for (model, d, first, n), out, (k, level) in zip(entries, outs, meta):
        single = ntbc.Model(d, model.weights, model.grid, model.grid_scale, model.grid_zero).infer(
            precision, first_block=first, n_blocks=n)
        assert torch.equal(out, single), f"material {k} level {level}"
    # oracle on a sample of every material's top level and its mip 2
    for (model, d, first, n), out, (k, level) in zip(entries, outs, meta):
        if level not in (0, 2):
            continue
        cfg, layers, g, _ = mats[k]
        mcfg = dataclasses.replace(cfg, blocks_w=d.blocks_w, blocks_h=d.blocks_h)
        lv = oracle_levels(mcfg, g)
        ids = np.unique(np.random.default_rng(k + 7 * level).integers(0, n, min(n, 400)))
        y_or = ON.heads(mcfg, lv, layers, ids + first, emu)
        w_or = ON.pack(y_or, mcfg.formats)
        single, heads = ntbc.Model(d, model.weights, model.grid, model.grid_scale, model.grid_zero).infer(
            precision, heads=True)
        hs = heads[torch.from_numpy(ids).cuda()].cpu().numpy()
        ws = u64(out[:, torch.from_numpy(ids).cuda()])
        res = OM.classify_differences(hs, ws, y_or, w_or, mcfg.formats)
        dy = np.abs(hs.astype(np.float64) - y_or).max()
        log(f"batch material {k} level {level}: identity {OM.identity(ws, w_or):.5f} max|dY| {dy:.3g} "
            f"differ {res['differ']} ties {res['ties']}")
        assert res["repack_exact"] and res["ties"] == res["differ"] and dy <= tol
    st = stamps.cpu().numpy()
    assert st[0] > 0 and (st[1:] >= st[0]).all()


def test_batch_graph_replay():
    mats = _materials()
    entries, _ = _entries(mats)
    batch = ntbc.Batch(entries, ntbc.BF16)
    eager = [o.clone() for o in batch.run()]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        batch.run()  # warm-up on the capture stream (kernel attributes set outside the capture)
        stream.synchronize()
        with torch.cuda.graph(g, stream=stream):
            batch.run()
    torch.cuda.current_stream().wait_stream(stream)
    for rep in range(3):
        for o in batch.outputs:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(batch.outputs, eager):
            assert torch.equal(o, e), f"replay {rep}"
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays


def test_fp8_batch_equals_single_launches():
    # FP8 E4M3 with each model's calibrated per-layer scales: the batch (staged epilogue for every
    # item) equals the single-range launches (register epilogue where an instance exists)
    mats = _materials()
    for _, _, _, model in mats:
        model.fp8_calibrate(4096)
    entries, meta = _entries(mats)
    batch = ntbc.Batch(entries, ntbc.FP8_E4M3)
    outs = batch.run()
    torch.cuda.synchronize()
    for (model, d, first, n), out, (k, level) in zip(entries, outs, meta):
        single = ntbc.Model(d, model.weights, model.grid, model.grid_scale, model.grid_zero)
        single.fp8_scales = model.fp8_scales
        assert torch.equal(out, single.infer(ntbc.FP8_E4M3, first_block=first, n_blocks=n)), f"material {k} level {level}"


def test_tile_shapes_give_the_same_blocks():
    # every BF16 kernel instance of the batch at 2, 4 and 8 waves per workgroup (the tile shapes the
    # autotuner chooses from): the blocks are those of the default shape, bit for bit
    mats = _materials()
    entries, meta = _entries(mats)
    batch = ntbc.Batch(entries, ntbc.BF16, tiles={})
    ref = [o.clone() for o in batch.run()]
    torch.cuda.synchronize()
    groups = batch.groups()
    assert len(groups) >= 3 and all(g["waves"] == 4 for g in groups)
    for w in (2, 8):
        for gi in range(len(groups)):
            batch.set_waves(gi, w)
        assert all(g["waves"] == w for g in batch.groups())
        for o in batch.outputs:
            o.zero_()
        outs = batch.run()
        torch.cuda.synchronize()
        for o, r, (k, level) in zip(outs, ref, meta):
            assert torch.equal(o, r), f"{w}-wave tiles: material {k} level {level}"
        log(f"{w}-wave tiles: {len(outs)} items equal")
    with pytest.raises(ntbc.NtbcError):
        batch.set_waves(0, 3)


def test_autotuner_picks_a_timed_shape():
    from paper_2407_09543_amd import autotune
    mats = _materials()
    entries, meta = _entries(mats)
    batch = ntbc.Batch(entries, ntbc.BF16, tiles={})
    table = autotune.tune(batch, reps=3)
    groups = batch.groups()
    assert len(table) == len(groups)
    for g in groups:
        t = table[autotune.key(g)]
        assert g["waves"] == t["waves"] == min(t["ms"], key=t["ms"].get)
    # a plan made with the table applies it
    again = ntbc.Batch(entries, ntbc.BF16, tiles={k: v["waves"] for k, v in table.items()})
    assert [g["waves"] for g in again.groups()] == [g["waves"] for g in groups]
