#!/usr/bin/env python3
"""NTBC benchmark on one MI355X: inference blocks/s of a five-texture 4096^2 material in BF16 and
FP32, with the decoded-PSNR delta between them, the reference-encoder and decoder rates, the encode
time of a material, the roofline position of the fused inference kernel, and the CPU oracle timed on
a bounded sample of the same workload.

A timed step is one inference of every block of the material (1,048,576 block positions x 5
textures = 5,242,880 BC blocks) with the inputs (grid, weights) resident in HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NTBC inference blocks/s at 4096² BF16 vs FP32 @ ΔPSNR≤0.1dB; encode s/material"
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP32_TFLOPS = 157.3
PEAK_FP8_TFLOPS = 5000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def flops_per_position(cfg):
    """Algorithmic FLOP of the MLP per block position: 2 * sum(fan_in * fan_out)."""
    return 2 * sum(i * o for i, o in cfg.layer_dims())


def psnr(a, b):
    from paper_2407_09543_amd import quality
    return quality.psnr(a, b)


def time_call(fn, steps, warmup, torch, settle_s=0.2):
    """Average ms per call over `steps` calls (HIP events on the current stream), after `warmup` calls
    and, untimed too, further calls until the GPU has been busy with this call for `settle_s` seconds
    (its clocks settle to the sustained rate of the workload)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0, n = time.perf_counter(), 0
    while time.perf_counter() - t0 < settle_s and n < 100000:
        for _ in range(8):
            fn()
        n += 8
        torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def cpu_baseline(cfg, layers, grid_codes, scale, zero, budget_s):
    """The FP64 oracle (heads and packing) on a sample of block positions, timed on the host."""
    from oracle import ntbc as ON
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # noqa: BLE001
        threads = 1
    levels = ON.grid_levels(cfg, codes=grid_codes, scales=scale, zeros=zero)
    rng = np.random.default_rng(0)
    n = 2048
    t_used = 0.0
    while True:
        ids = rng.choice(cfg.n_positions, n, replace=False)
        t0 = time.perf_counter()
        ON.infer_blocks(cfg, levels, layers, ids)
        t_used = time.perf_counter() - t0
        if t_used * 2 > budget_s or 2 * n > cfg.n_positions:
            break
        n *= 2
    blocks = n * len(cfg.formats)
    info = {"value": blocks / t_used, "unit": "blocks/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} random block positions of the 4096^2 five-texture material "
                      f"({blocks} BC blocks), FP64 heads + packing, {t_used:.1f} s"}
    return info, ids, ON.infer_blocks(cfg, levels, layers, ids)[0]


def cpu_legs(cfg, layers, grid_codes, scale, zero, mat, n_sample):
    """The other oracle timings, each bounded to a few seconds: the inference sample again on one core,
    oracle training (100 steps of the 256^2 two-texture config at batch 512; one step of the 1024^2
    five-texture config at batch 16,384) and the reference encoder (both small materials in full, one
    texture of the 4096^2 material on a 65,536-block sample)."""
    import dataclasses
    from oracle import bc as OB
    from oracle import ntbc as ON
    from paper_2407_09543_amd import synth
    from threadpoolctl import threadpool_limits
    out = {}
    levels = ON.grid_levels(cfg, codes=grid_codes, scales=scale, zeros=zero)
    n1 = min(65536, max(4096, n_sample // 4))
    ids = np.random.default_rng(1).choice(cfg.n_positions, n1, replace=False)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ON.infer_blocks(cfg, levels, layers, ids)
        dt = time.perf_counter() - t0
    out["inference_one_core"] = {"value": n1 * len(cfg.formats) / dt, "unit": "blocks/s", "cores": 1,
                                 "sample": f"{n1} random block positions of the 4096^2 material, {dt:.1f} s"}

    def encode_ref(blocks, fmt):
        return OB.bc1_encode_ref(blocks) if fmt == 1 else OB.bc4_encode_ref(blocks[..., 0])

    def training(c, m, seed, steps, batch, total):
        blocks = [OB.image_to_blocks(t.texels) for t in m.textures]
        t0 = time.perf_counter()
        ref = [encode_ref(b, t.fmt) for b, t in zip(blocks, m.textures)]
        t_enc = time.perf_counter() - t0
        tg = ON.Targets(c.formats, ref, blocks)
        st = ON.TrainState(synth.init_grid(c, seed), synth.init_weights(c, seed))
        t0 = time.perf_counter()
        for s in range(steps):
            ON.train_step(c, st, tg, synth.batch_ids(seed, s, batch, c.n_positions), s, total, False)
        return (time.perf_counter() - t0) / steps, t_enc, sum(len(b) for b in blocks)

    c1 = synth.config_small(256)
    ms1, enc1, nb1 = training(c1, synth.material_small(256, 1), 1, 100, 512, 100)
    c2 = dataclasses.replace(synth.config_mid(1024), grid_u8=False)
    ms2, enc2, nb2 = training(c2, synth.material_five(1024, 2), 2, 1, 16384, 2200)
    out["training"] = {"ms_per_step_256_two_texture_batch_512": ms1 * 1e3,
                       "ms_per_step_1024_five_texture_batch_16384": ms2 * 1e3, "unit": "ms/step (FP64 oracle)"}
    tex = mat.textures[0]
    sample = OB.image_to_blocks(tex.texels)[np.random.default_rng(2).choice(cfg.n_positions, 65536, replace=False)]
    t0 = time.perf_counter()
    encode_ref(sample, tex.fmt)
    enc3 = time.perf_counter() - t0
    out["ref_encoder"] = {"blocks_per_s_256_material": nb1 / enc1, "blocks_per_s_1024_material": nb2 / enc2,
                          "blocks_per_s_4096_bc1_sample": 65536 / enc3,
                          "note": "the 4096^2 figure is from 65,536 blocks of the diffuse texture"}
    return out


def versus_oracle(cfg, mat, outs, ids, words_or, names):
    """Block identity and decoded-PSNR delta of every precision's blocks against the FP64 oracle's, on
    the oracle's sample of block positions (all of them when the sample covers the material): PSNR of
    the sampled blocks' decoded texels against the texture, both sides decoded by the oracle's decoder."""
    from oracle import bc as OB
    from paper_2407_09543_amd import quality
    orig = [OB.image_to_blocks(m.texels)[ids] for m in mat.textures]

    def decode(t, words):
        return OB.bc1_decode(words) if cfg.formats[t] == 1 else OB.bc4_decode(words)[..., None]

    sse_or = [quality.squared_error(decode(t, words_or[t]), orig[t]) for t in range(len(cfg.formats))]
    n_vals = [o.size for o in orig]
    psnr_or = [quality.psnr_from_sse(e, n) for e, n in zip(sse_or, n_vals)]
    mat_or = quality.psnr_from_sse(sum(sse_or), sum(n_vals))
    out = {"positions": int(len(ids)), "psnr_db_oracle": psnr_or, "psnr_db_material_oracle": mat_or}
    for prec, name in names.items():
        w = outs[prec][:, ids].cpu().numpy().view(np.uint64)
        sse = [quality.squared_error(decode(t, w[t]), orig[t]) for t in range(len(cfg.formats))]
        ps = [quality.psnr_from_sse(e, n) for e, n in zip(sse, n_vals)]
        d = [abs(a - b) if np.isfinite(a) and np.isfinite(b) else (0.0 if a == b else float("inf"))
             for a, b in zip(ps, psnr_or)]
        dm = abs(quality.psnr_from_sse(sum(sse), sum(n_vals)) - mat_or)
        out[name] = {"identity": float((w == words_or).mean()),
                     "identity_per_texture": [float((w[t] == words_or[t]).mean()) for t in range(len(cfg.formats))],
                     "dpsnr_db": {"per_texture": d, "max": max(d), "material": dm},
                     "gate_dpsnr_0p1db": bool(max(d) <= 0.1 and dm <= 0.1)}
    return out


def traffic_from_profile(path, kernel_src):
    """HBM bytes per launch of the inference kernel from a committed counter summary, or None if the
    summary is missing or was taken on a different kernel source (the sha256 of the kernel's source
    files, concatenated in order, is recorded in it)."""
    import hashlib
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for src in kernel_src:  # the kernel's sources, in order
        with open(src, "rb") as fh:
            h.update(fh.read())
    digest = h.hexdigest()
    if fields.get("kernel_source_sha256") != digest or "hbm_bytes_per_launch" not in fields:
        return None
    return float(fields["hbm_bytes_per_launch"])


def copy_probe(torch, mib=1024, reps=5):
    """A plain device-to-device copy of known size, for scaling the FETCH_SIZE/WRITE_SIZE counters."""
    src = torch.empty(mib << 20, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read_per_launch": mib << 20, "launches": reps}), flush=True)


def batched_decode(torch, ntbc, synth, reps=10):
    """Load-time decode of 16 materials with full mip chains (sizes 512..4096, MLP widths 64..256,
    3-5 textures, random parameters of those shapes): one batched BF16 launch per kernel instance,
    replayed from a HIP graph, against per-material FP32 launches of the same block grids (and, for
    context, per-material BF16 launches)."""
    from paper_2407_09543_amd import autotune
    dev = torch.device("cuda:0")
    entries, mat_of, per_mat = autotune.batched_decode_workload()
    n_blocks = sum(e[1].n_textures * e[3] for e in entries)
    batch = ntbc.Batch(entries, ntbc.BF16)  # tile shapes from the committed autotuner table
    tile_shapes = {autotune.key(g): g["waves"] for g in batch.groups()}
    stamps = torch.zeros(len(entries) + 1, dtype=torch.int64, device=dev)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        batch.run(stamps)
        stream.synchronize()
        with torch.cuda.graph(graph, stream=stream):
            batch.run(stamps)
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    ms_batch = time_call(graph.replay, reps, 2, torch)
    graph.replay()
    torch.cuda.synchronize()
    st = stamps.cpu().numpy().astype(np.float64)
    ticks = st[1:] - st[0]
    lat_us = [0.01 * max(ticks[i] for i in range(len(entries)) if mat_of[i] == m) for m in range(16)]
    # per-material launches, one single-range launch per mip (weights packed once per mip model, then
    # reused), in FP32 (the comparison asked for) and in BF16 (the same kernels as the batch, unbatched)
    outs = [[torch.empty((mp.desc.n_textures, mp.desc.blocks_w * mp.desc.blocks_h), dtype=torch.int64, device=dev)
             for mp in mips] for mips in per_mat]

    def sequence(prec):
        for mips, o in zip(per_mat, outs):
            for mp, oo in zip(mips, o):
                mp.infer(prec, out=oo)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(17)]
        ev[0].record()
        for m, (mips, o) in enumerate(zip(per_mat, outs)):
            for mp, oo in zip(mips, o):
                mp.infer(prec, out=oo, reuse_packed=True)
            ev[m + 1].record()
        torch.cuda.synchronize()
        total = ev[0].elapsed_time(ev[16])
        lat = [ev[0].elapsed_time(ev[m + 1]) * 1e3 for m in range(16)]
        return {"ms": total, "blocks_per_s": n_blocks / (total * 1e-3),
                "latency_us_p50": float(np.percentile(lat, 50)), "latency_us_p99": float(np.percentile(lat, 99))}

    per_fp32 = sequence(ntbc.FP32)
    per_bf16 = sequence(ntbc.BF16)
    return {"workload": "16 materials 512^2..4096^2 with full mip chains, widths 64..256, 3-5 textures",
            "items": len(entries), "blocks": n_blocks,
            "batched_bf16_graph": {"ms": ms_batch, "blocks_per_s": n_blocks / (ms_batch * 1e-3),
                                   "latency_us_p50": float(np.percentile(lat_us, 50)),
                                   "latency_us_p99": float(np.percentile(lat_us, 99)),
                                   "stamp_span_us": float(0.01 * ticks.max())},
            "tile_waves": tile_shapes, "tile_table": autotune.TABLE_PATH if os.path.exists(autotune.TABLE_PATH) else None,
            "per_material_fp32": per_fp32, "per_material_bf16": per_bf16,
            "latency_note": "batched: completion of a material's last mip since the batch start (100 MHz "
                            "real-time counter); per-material: completion since the first launch of the "
                            "sequence (one launch per mip)"}


def _finite(x):
    """Replaces infinite or NaN floats (PSNR of an exact texture) by None: strict JSON has neither."""
    if isinstance(x, dict):
        return {k: _finite(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_finite(v) for v in x]
    if isinstance(x, (float, np.floating)) and not np.isfinite(x):
        return None
    return x


def _plain(x):
    """JSON fallback for NumPy scalars."""
    if isinstance(x, np.generic):
        return x.item()
    raise TypeError(f"not JSON serializable: {type(x).__name__}")


def paper_layout(args):
    """The paper's own network layout (endpoint network + per-texel colour network, SELU, half precision)
    on the workload of its inference table: a 4096^2 material of two BC1 and four BC4 textures, and one
    of two BC1 textures only, each with the aggressive (one model) and the conservative (a BC1 model
    and a BC4 model) layout; random parameters of the paper's shapes (the cost does not depend on the
    values).  Times one full material per call (weight packing included)."""
    import torch
    from paper_2407_09543_amd import ntbc
    rng = np.random.default_rng(11)
    dev = torch.device("cuda:0")
    bw = bh = args.size // 4

    def model(formats):
        e = sum(6 if f == 1 else 2 for f in formats)
        c = sum(3 if f == 1 else 1 for f in formats)

        def net(n_in, n_out):
            dims = [n_in, 64, 64, 64, n_out]
            return np.concatenate([np.concatenate([(rng.standard_normal((dims[k + 1], dims[k])) * np.sqrt(2.0 / dims[k])).ravel(),
                                                   0.2 * rng.standard_normal(dims[k + 1])]) for k in range(4)]).astype(np.float32)

        def grid(levels):
            nv = sum((16 << l) ** 2 for l in range(levels))
            return (torch.from_numpy(rng.integers(0, 256, (nv, 2), dtype=np.uint8)).to(dev),
                    torch.full((levels,), 0.006, dtype=torch.float32, device=dev),
                    torch.full((levels,), 128, dtype=torch.int32, device=dev))

        eg, es, ez = grid(7)
        cg, cs, cz = grid(8)
        return ntbc.FaithfulModel(formats, bw, bh, eg, cg, torch.from_numpy(net(14, e)).to(dev),
                                  torch.from_numpy(net(16, c)).to(dev), ep_scale=es, ep_zero=ez, col_scale=cs,
                                  col_zero=cz)

    def flop(formats):
        e = sum(6 if f == 1 else 2 for f in formats)
        c = sum(3 if f == 1 else 1 for f in formats)
        return 2 * ((14 * 64 + 2 * 64 * 64 + 64 * e) + 16 * (16 * 64 + 2 * 64 * 64 + 64 * c)) * bw * bh

    out = {"texture_size": args.size, "blocks_per_texture": bw * bh,
           "paper_ms_rx7900xt_half": {"bc1_bc4_conservative": 49.84, "bc1_only_conservative": 25.57,
                                      "bc1_bc4_aggressive": 27.31, "bc1_only_aggressive": 25.96,
                                      "note": "Tab. inferPerf: another GPU; context only"}}
    for name, formats in (("bc1_bc4", [1, 1, 4, 4, 4, 4]), ("bc1_only", [1, 1])):
        for layout in ("aggressive", "conservative"):
            groups = [formats] if layout == "aggressive" else [g for g in ([f for f in formats if f == 1],
                                                                          [f for f in formats if f == 4]) if g]
            models = [model(g) for g in groups]
            outs = [torch.empty((len(g), bw * bh), dtype=torch.int64, device=dev) for g in groups]
            ms = time_call(lambda: [m.infer(out=o) for m, o in zip(models, outs)], args.steps, args.warmup, torch)
            fl = sum(flop(g) for g in groups)
            out[f"{name}_{layout}"] = {"ms": ms, "blocks_per_s": len(formats) * bw * bh / (ms * 1e-3),
                                       "models": len(groups), "tflops": fl / (ms * 1e-3) / 1e12,
                                       "frac_fp16_peak": fl / (ms * 1e-3) / PEAK_BF16_TFLOPS / 1e12}
    out["training"] = paper_layout_training(args, rng, bw, bh)
    return out


def paper_layout_training(args, rng, bw, bh):
    """Training steps of the paper's layout (ntbc_faithful_train_step, FP32 products) for the two-BC1 +
    four-BC4 4096^2 material at the encode's batch of blocks (the colour network sees 16 texels each),
    aggressive (one model) and conservative (two models, one step each); random textures and
    parameters (the cost does not depend on the values)."""
    import torch
    from paper_2407_09543_amd import ntbc
    dev = torch.device("cuda:0")
    six = [1, 1, 4, 4, 4, 4]
    tex = [torch.from_numpy(rng.integers(0, 256, (args.size, args.size, 3) if f == 1 else (args.size, args.size),
                                         dtype=np.uint8)).to(dev) for f in six]
    ref = [ntbc.encode_ref(t, f) for t, f in zip(tex, six)]

    def net(n_in, n_out):
        dims = [n_in, 64, 64, 64, n_out]
        return torch.from_numpy(np.concatenate([np.concatenate([
            (rng.standard_normal((dims[k + 1], dims[k])) * np.sqrt(1.0 / dims[k])).ravel(),
            0.1 * rng.standard_normal(dims[k + 1])]) for k in range(4)]).astype(np.float32)).to(dev)

    def grid(levels):
        nv = sum((16 << l) ** 2 for l in range(levels))
        return torch.from_numpy(rng.uniform(-0.1, 0.1, (nv, 2)).astype(np.float32)).to(dev)

    out = {"batch_blocks": args.batch, "texels_per_step": 16 * args.batch,
           "paper_minutes_20k_iterations": {"aggressive": 10, "conservative": 16,
                                            "note": "Fig. training: another GPU and batch; context only"}}
    ids = ntbc.batch_ids(3, 0, args.batch, bw * bh)
    for layout, groups in (("aggressive", [list(range(6))]), ("conservative", [[0, 1], [2, 3, 4, 5]])):
        trainers = []
        for g in groups:
            fm = [six[i] for i in g]
            e = sum(6 if f == 1 else 2 for f in fm)
            c = sum(3 if f == 1 else 1 for f in fm)
            tg = ntbc.Targets(torch.stack([ref[i] for i in g]), [tex[i] for i in g])
            trainers.append(ntbc.FaithfulTrainer(fm, bw, bh, grid(7), grid(8), net(14, e), net(16, c), tg, args.batch,
                                                 20000))
        step = [0]

        def run():
            for tr in trainers:
                tr.step(ids, step[0])
            step[0] += 1
        ms = time_call(run, 10, 2, torch)
        out[layout] = {"ms_per_step": ms, "models": len(groups), "minutes_20k_iterations": ms * 20000 / 60000.0}
        del trainers
        torch.cuda.empty_cache()
    return out


def naive_ablation(args, cfg, tex, ntbc_psnr):
    """The naive approach (Sec. 3.1: weight head, two-stage 80/20 training) encoded with the same
    steps, batch, seed and training precision as NTBC, its blocks inferred in BF16: PSNR per texture
    beside NTBC's, its model size, and its train step and inference times."""
    import dataclasses
    import torch
    from paper_2407_09543_amd import encode, ntbc
    ncfg = dataclasses.replace(cfg, variant="naive")
    log(f"naive ablation: {args.encode_steps} steps + 10% QAT")
    res = encode.encode_material(tex, ncfg, steps=args.encode_steps, batch=args.batch, seed=3,
                                 precision=ntbc.BF16, train_precision=ntbc.PRECISIONS[args.train_precision])
    p = encode.psnr_of_words(res.ntbc_words, tex, cfg.formats, args.size)
    out = torch.empty_like(res.ntbc_words)
    ms = time_call(lambda: res.model.infer(ntbc.BF16, out=out, reuse_packed=True), 10, 2, torch)
    return {"psnr_db_naive": p, "psnr_db_ntbc": ntbc_psnr,
            "ntbc_minus_naive_db": [None if a is None or b is None else a - b for a, b in zip(ntbc_psnr, p)],
            "model_bytes_bf16_weights": encode.model_bytes(ncfg, 2), "head_dim": ncfg.head_dim,
            "stage2_from_step": (4 * res.steps) // 5, "steps": res.steps,
            "ms_per_train_step": res.train_seconds * 1e3 / res.steps,
            "inference_ms_bf16": ms, "inference_blocks_per_s": res.ntbc_words.numel() / (ms * 1e-3),
            "note": "the naive model's inference takes the LDS-staged epilogue (no register-resident instance)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--encode-steps", type=int, default=20000,
                    help="base training steps of the encode (plus 10%% with grid QAT)")
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--kappa", type=float, default=4.0, help="judge: fall back when SSE > kappa * SSE_ref")
    ap.add_argument("--train-precision", choices=("bf16", "fp32"), default="bf16",
                    help="operands of the training products (FP32 accumulation and master parameters either way)")
    ap.add_argument("--no-encode", action="store_true",
                    help="skip the encode; time inference on random parameters of the same shape")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched multi-material decode")
    ap.add_argument("--no-naive", action="store_true", help="skip the naive-approach ablation encode")
    ap.add_argument("--no-paper-layout", action="store_true",
                    help="skip the paper's own network layout (its inference table and training steps)")
    ap.add_argument("--copy-probe", action="store_true", help="only run the counter-calibration copy")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(inference shards by block range with no communication between GPUs)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_09543_amd import encode, ntbc, quality, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe:
        copy_probe(torch)
        return
    dev = torch.device("cuda:0")
    cfg = synth.config_paper_scale(args.size)
    log(f"generating {args.size}^2 five-texture material")
    mat = synth.material_five(args.size, 3)
    tex = [torch.from_numpy(t.texels).to(dev) for t in mat.textures]

    # reference encoding of the targets (also the fallback), and decode
    ref = [ntbc.encode_ref(t, f) for t, f in zip(tex, cfg.formats)]
    enc_ms = time_call(lambda: [ntbc.encode_ref(t, f) for t, f in zip(tex, cfg.formats)], 3, 1, torch)
    dec_ms = time_call(lambda: [ntbc.decode(r, args.size, args.size, f) for r, f in zip(ref, cfg.formats)],
                       5, 1, torch)
    ref_psnr = [psnr(ntbc.decode(r, args.size, args.size, f).cpu().numpy(), t.texels)
                for r, f, t in zip(ref, cfg.formats, mat.textures)]

    encode_info = None
    if args.no_encode:
        # random parameters of the paper-scale shape (inference cost does not depend on values)
        layers = synth.init_weights(cfg, 3)
        rng = np.random.default_rng(3)
        layers = [(w, (0.3 * rng.standard_normal(len(b))).astype(np.float32)) for w, b in layers]
        codes, _, _ = synth.random_u8_grid(cfg, 3)
        scale = (np.full(cfg.n_levels, 0.7 / 128.0)).astype(np.float32)
        zero = np.full(cfg.n_levels, 128, dtype=np.int32)
        model = ntbc.Model(ntbc.desc_from_config(cfg), torch.from_numpy(synth.flatten_weights(layers)).to(dev),
                           torch.from_numpy(codes).to(dev), torch.from_numpy(scale).to(dev),
                           torch.from_numpy(zero).to(dev))
        model_note = "random parameters of the paper-scale shape (inference cost does not depend on values)"
    else:
        log(f"encoding the material: {args.encode_steps} steps + 10% QAT at batch {args.batch}, "
            f"{args.train_precision} training products")
        res = encode.encode_material(tex, cfg, steps=args.encode_steps, batch=args.batch, seed=3,
                                     precision=ntbc.BF16, kappa=args.kappa, delta=0.0,
                                     train_precision=ntbc.PRECISIONS[args.train_precision])
        model = res.model
        layers = synth.unflatten_weights(cfg, res.weights.cpu().numpy())
        codes = model.grid.cpu().numpy()
        scale = model.grid_scale.cpu().numpy()
        zero = model.grid_zero.cpu().numpy()
        ntbc_psnr = encode.psnr_of_words(res.ntbc_words, tex, cfg.formats, args.size)
        judged_psnr = encode.psnr_of_words(res.words, tex, cfg.formats, args.size)
        bc_bytes = 8 * cfg.n_positions * len(cfg.formats)
        encode_info = {
            "seconds": res.seconds, "train_seconds": res.train_seconds, "steps": res.steps, "batch": args.batch,
            "train_precision": args.train_precision,
            "ms_per_train_step": res.train_seconds * 1e3 / res.steps,
            "includes": "reference encode of the targets, all training steps, grid quantisation, BF16 "
                        "inference, per-block judge; textures already in HBM",
            "psnr_db_ntbc": ntbc_psnr, "psnr_db_after_judge": judged_psnr, "psnr_db_ref_encoder": ref_psnr,
            "ssim_central_1024": {"ntbc": encode.ssim_of_words(res.ntbc_words, tex, cfg.formats, args.size),
                                  "after_judge": encode.ssim_of_words(res.words, tex, cfg.formats, args.size),
                                  "ref_encoder": encode.ssim_of_words(torch.stack(ref), tex, cfg.formats, args.size)},
            "judge": {"kappa": args.kappa, "delta": 0.0, "fallback_blocks": res.fallback_blocks,
                      "exception_list_bytes": sum(encode.exception_list_bytes(c, cfg.n_positions)
                                                  for c in res.fallback_blocks)},
            "model_bytes_bf16_weights": encode.model_bytes(cfg, 2), "bc_bytes": bc_bytes,
            "total_bytes_after_judge": encode.model_bytes(cfg, 2) + sum(
                encode.exception_list_bytes(c, cfg.n_positions) for c in res.fallback_blocks),
            "judge_sweep": encode.judge_sweep(res.ntbc_words, res.ref_words, tex, cfg.formats, args.size,
                                              encode.model_bytes(cfg, 2)),
            "storage_matched_baseline": {"what": "reference BC of the 2x2-averaged texture, nearest upsampled",
                                         "bytes": bc_bytes // 4,
                                         "psnr_db": encode.downsampled_ref_psnr(tex, cfg.formats, args.size)},
        }
        model_note = "parameters trained by the encode above"
        if not args.no_naive:
            encode_info["naive_ablation"] = naive_ablation(args, cfg, tex, ntbc_psnr)
    n_blocks = cfg.n_positions * len(cfg.formats)
    # FP8 E4M3 scales from a 65,536-block calibration sample (not part of the timed inference)
    torch.cuda.synchronize()
    t_cal = time.perf_counter()
    model.fp8_calibrate(65536)
    torch.cuda.synchronize()
    calib_ms = (time.perf_counter() - t_cal) * 1e3
    outs = {}
    for prec in (ntbc.BF16, ntbc.FP16, ntbc.FP8_E4M3, ntbc.FP32):
        outs[prec] = torch.empty((len(cfg.formats), cfg.n_positions), dtype=torch.int64, device=dev)
        model.infer(prec, out=outs[prec])
    torch.cuda.synchronize()
    out_bf, out_fp = outs[ntbc.BF16], outs[ntbc.FP32]

    log(f"timing BF16 inference: {args.steps} steps after {args.warmup} warm-up")
    ms_bf = time_call(lambda: model.infer(ntbc.BF16, out=out_bf, reuse_packed=True), args.steps, args.warmup, torch)
    model.infer(ntbc.FP16, out=outs[ntbc.FP16])
    ms_h = time_call(lambda: model.infer(ntbc.FP16, out=outs[ntbc.FP16], reuse_packed=True), args.steps,
                     args.warmup, torch)
    model.infer(ntbc.FP8_E4M3, out=outs[ntbc.FP8_E4M3])
    ms_f8 = time_call(lambda: model.infer(ntbc.FP8_E4M3, out=outs[ntbc.FP8_E4M3], reuse_packed=True), args.steps,
                      args.warmup, torch)
    model.infer(ntbc.FP32, out=out_fp)
    steps_fp = max(2, args.steps // 4)
    ms_fp = time_call(lambda: model.infer(ntbc.FP32, out=out_fp, reuse_packed=True), steps_fp, 1, torch)

    # quality: decoded PSNR of every precision's blocks against the texture, and deltas to FP32
    sq_err = {}
    psnrs = {}
    for prec, words in outs.items():
        psnrs[prec], sq_err[prec] = [], 0.0
        for t, (f, m) in enumerate(zip(cfg.formats, mat.textures)):
            dec = ntbc.decode(words[t].contiguous(), args.size, args.size, f).cpu().numpy()
            e = quality.squared_error(dec, m.texels)
            psnrs[prec].append(quality.psnr_from_sse(e, m.texels.size))
            sq_err[prec] += e
    n_values = sum(m.texels.size for m in mat.textures)

    def material_psnr(prec):
        return quality.psnr_from_sse(sq_err[prec], n_values)

    def versus_fp32(prec):
        d = [abs(a - b) for a, b in zip(psnrs[prec], psnrs[ntbc.FP32])]
        return {"identity_vs_fp32": float((outs[prec] == out_fp).float().mean().item()),
                "dpsnr_db_vs_fp32": {"per_texture": d, "max": max(d),
                                     "material": abs(material_psnr(prec) - material_psnr(ntbc.FP32))}}

    identity = versus_fp32(ntbc.BF16)["identity_vs_fp32"]
    psnr_bf, psnr_fp = psnrs[ntbc.BF16], psnrs[ntbc.FP32]

    flop = flops_per_position(cfg) * cfg.n_positions
    achieved = flop / (ms_bf * 1e-3) / 1e12
    traffic = traffic_from_profile(os.path.join(ROOT, "profiles", "k_infer_lds_bf16_4096_five_texture_traffic.txt"),
                                   [os.path.join(ROOT, "paper_2407_09543_amd", "csrc", f)
                                    for f in ("infer.hip", "device.h")])
    result = {
        "metric": METRIC,
        "value": n_blocks / (ms_bf * 1e-3),
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_bf,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"ntbc-inference-{args.size}x{args.size}-five-texture",
                   "texture_size": args.size, "textures": "2xBC1+3xBC4", "block_positions": cfg.n_positions,
                   "blocks_per_step": n_blocks, "mlp": "64-256x3-162 relu/sigmoid",
                   "grid": "8 levels 8..1024 x 8 uint8", "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16_TFLOPS, "traffic": traffic,
                     "kernel": "k_infer_lds<BF16,256,4,2,2,3>", "flop_per_launch": flop,
                     "note": "priced against the BF16 matrix-core peak; the kernel is limited by its vector-ALU "
                             "work (exact float32 nearest-palette searches, sigmoid, grid gather): "
                             "profiles/k_infer_lds_bf16_4096_five_texture_counters.txt"},
        "fp32": {"blocks_per_s": n_blocks / (ms_fp * 1e-3), "ms_per_step": ms_fp,
                 "tflops": flop / (ms_fp * 1e-3) / 1e12, "frac_fp32_peak": flop / (ms_fp * 1e-3) / 1e12 / PEAK_FP32_TFLOPS},
        "speedup_bf16_vs_fp32": ms_fp / ms_bf,
        "identity_bf16_vs_fp32": identity,
        "dpsnr_db_bf16_vs_fp32": versus_fp32(ntbc.BF16)["dpsnr_db_vs_fp32"],
        "psnr_db_bf16": psnr_bf, "psnr_db_fp32": psnr_fp,
        "fp16": dict({"blocks_per_s": n_blocks / (ms_h * 1e-3), "ms_per_step": ms_h,
                      "frac_fp16_peak": flop / (ms_h * 1e-3) / 1e12 / PEAK_BF16_TFLOPS,
                      "psnr_db": psnrs[ntbc.FP16]}, **versus_fp32(ntbc.FP16)),
        "fp8_e4m3": dict({"blocks_per_s": n_blocks / (ms_f8 * 1e-3), "ms_per_step": ms_f8,
                          "frac_fp8_peak": flop / (ms_f8 * 1e-3) / 1e12 / PEAK_FP8_TFLOPS,
                          "calibration_ms": calib_ms, "scales": model.fp8_scales.cpu().numpy().tolist(),
                          "psnr_db": psnrs[ntbc.FP8_E4M3]}, **versus_fp32(ntbc.FP8_E4M3)),
        "psnr_db_material": {"bf16": material_psnr(ntbc.BF16), "fp16": material_psnr(ntbc.FP16),
                             "fp8_e4m3": material_psnr(ntbc.FP8_E4M3), "fp32": material_psnr(ntbc.FP32)},
        "gate_dpsnr_0p1db": {p: {"per_texture": bool(versus_fp32(v)["dpsnr_db_vs_fp32"]["max"] <= 0.1),
                                 "material": bool(versus_fp32(v)["dpsnr_db_vs_fp32"]["material"] <= 0.1)}
                             for p, v in (("bf16", ntbc.BF16), ("fp16", ntbc.FP16), ("fp8_e4m3", ntbc.FP8_E4M3))},
        "ref_encoder": {"ms_per_material": enc_ms, "blocks_per_s": n_blocks / (enc_ms * 1e-3), "psnr_db": ref_psnr},
        "decoder": {"ms_per_material": dec_ms, "blocks_per_s": n_blocks / (dec_ms * 1e-3)},
        "encode_s_per_material": encode_info["seconds"] if encode_info else None,
        "encode": encode_info,
        "model_note": model_note,
    }
    log("the paper's own network layout on its inference-table workload")
    if not args.no_paper_layout:
        result["paper_layout"] = paper_layout(args)
    if not args.no_batched:
        log("batched load-time decode of 16 materials with mip chains")
        result["batched_decode"] = batched_decode(torch, ntbc, synth)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        result["cpu_baseline"], ids_or, words_or = cpu_baseline(cfg, layers, codes, scale, zero, args.cpu_seconds)
        log("oracle legs: one core, training, reference encoder")
        result["cpu_baseline"]["legs"] = cpu_legs(cfg, layers, codes, scale, zero, mat, len(ids_or))
        log("identity and decoded-PSNR delta of every precision against the FP64 oracle")
        result["vs_fp64_oracle"] = versus_oracle(
            cfg, mat, outs, ids_or, words_or,
            {ntbc.BF16: "bf16", ntbc.FP16: "fp16", ntbc.FP8_E4M3: "fp8_e4m3", ntbc.FP32: "fp32"})
    result["paper_context"] = {
        "hardware": "one Radeon RX 7900 XT, half precision (other GPU, network and material)",
        "inference_ms_six_textures_4096": 27.31, "inference_blocks_per_s": 6291456 / 27.31e-3,
        "encode_minutes_per_material_20000_iterations": 10, "source": "Tab. inferPerf; Fig. training"}
    result["note"] = "a PSNR of null means zero error (lossless)"
    print(json.dumps(_finite(result), default=_plain, allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
