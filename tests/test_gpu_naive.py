"""GPU parity of the naive approach (Sec. 3.1; model variant NTBC_NAIVE) against its oracle.

Inference: the weight-head pack is bit-exact (the oracle's float32 packer on the kernel's own heads
reproduces every word) in FP32, BF16 and FP16, single range, batched and allocation-free.  Training:
the two-stage loss and its head gradients within float32 rounding of the oracle; stage-1 gradients of
a whole train step within 1e-4 of the FP64 oracle; a stage-2 step leaves every parameter but the
endpoint head's rows of the last layer (and their moments) bit-identical, and moves those rows as the
oracle's Adam does."""
import dataclasses

import numpy as np
import pytest
import torch

from cases import TrainProblem
from util import ensure_built, log, u64
from oracle import naive as NV
from oracle import ntbc as ON
from paper_2407_09543_amd import ntbc, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    assert torch.cuda.is_available()


def _problem(which, seed=1):
    if which == "small":
        cfg = dataclasses.replace(synth.config_small(256), variant="naive")
        return TrainProblem(cfg, synth.material_small(256, seed), seed)
    cfg = dataclasses.replace(synth.config_mid(256), grid_u8=False, variant="naive")
    return TrainProblem(cfg, synth.material_five(256, seed), seed)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_head_dim_of_the_weight_head():
    pb = _problem("mid")
    nw, hd, _ = ntbc.model_sizes(pb.desc)
    # five textures: endpoints 2*6 + 3*2 = 18, weights 16 * 5 = 80
    assert hd == 98 == pb.cfg.head_dim == NV.NaiveLayout(pb.cfg.formats).H
    assert nw == pb.cfg.n_weights


@pytest.mark.parametrize("which", ["small", "mid"])
@pytest.mark.parametrize("precision", [ntbc.FP32, ntbc.BF16, ntbc.FP16])
def test_pack_bit_exact_on_kernel_heads(which, precision):
    pb = _problem(which, 2)
    model = ntbc.Model(pb.desc, pb.flat_d, pb.grid_d)
    n = pb.cfg.n_positions - 37                          # ragged last tile
    words, heads = model.infer(precision, first_block=11, n_blocks=n, heads=True)
    words = u64(words)
    h = heads.cpu().numpy()
    ref = NV.pack(h, pb.cfg.formats)
    assert np.array_equal(words, ref)
    if precision == ntbc.FP32:
        y_or = ON.heads(pb.cfg, ON.grid_levels(pb.cfg, grid=pb.grid), pb.layers, np.arange(11, 11 + n))
        dy = float(np.abs(h - y_or).max())
        log(f"naive {which} fp32: max|dY| {dy:.3g}")
        assert dy <= 1e-5
    # the noalloc entry point and the batched decode run the same epilogue
    w2 = u64(model.infer_noalloc(precision, first_block=11, n_blocks=n))
    assert np.array_equal(w2, words)
    if precision != ntbc.FP32:
        b = ntbc.Batch([(model, pb.desc, 11, n)], precision)
        b.run()
        torch.cuda.synchronize()
        assert np.array_equal(u64(b.outputs[0]), words)


@pytest.mark.parametrize("which", ["small", "mid"])
@pytest.mark.parametrize("stage", [1, 2])
def test_loss_and_head_gradients(which, stage):
    # heads uniform in (0, 1) at 3,000 positions (a ragged last group of 16); both sides take the same
    # float32 heads, so the stage-2 weight choices agree exactly; the rest is float32 rounding
    pb = _problem(which, 3)
    rng = np.random.default_rng(4)
    ids, ids_d = pb.ids(5, 3000)
    y = rng.uniform(0.0, 1.0, (len(ids), pb.cfg.head_dim)).astype(np.float32)
    losses, dh = ntbc.naive_loss_grad(pb.desc, pb.tg_gpu, torch.from_numpy(y).cuda(), ids_d, stage)
    l_or, g_or = NV.loss_and_grad(y.astype(np.float64), pb.tg_oracle, ids, stage)
    losses = losses.cpu().numpy()
    dh = dh.cpu().numpy()
    log(f"naive loss {which} stage {stage}: gpu {losses[0]:.7g} oracle {l_or:.7g}; rel grad {_rel(dh, g_or):.3g}")
    assert abs(losses[0] - l_or) <= 1e-5 * l_or
    assert (losses[1:4] == 0).all() and losses[4] == 0
    assert _rel(dh, g_or) <= 1e-5
    E = NV.NaiveLayout(pb.cfg.formats).E
    if stage == 2:
        assert (dh[:, E:] == 0).all()


def test_loss_rejects_bad_stage_and_variant():
    pb = _problem("small")
    ids, ids_d = pb.ids(1, 16)
    y = torch.rand((16, pb.cfg.head_dim), device="cuda")
    with pytest.raises(ntbc.NtbcError):
        ntbc.naive_loss_grad(pb.desc, pb.tg_gpu, y, ids_d, 3)
    d = ntbc.desc_from_config(dataclasses.replace(pb.cfg, variant="ntbc"))
    with pytest.raises(ntbc.NtbcError):
        ntbc.naive_loss_grad(d, pb.tg_gpu, y, ids_d, 1)


@pytest.mark.parametrize("precision", [ntbc.FP32, ntbc.BF16])
def test_train_step_stage1_gradients(precision):
    pb = _problem("mid", 6)
    ids, ids_d = pb.ids(7, 2048)
    tr = ntbc.Trainer(pb.desc, pb.grid_d, pb.flat_d, pb.tg_gpu, 2048, 100, precision=precision)
    losses = tr.step(ids_d, 0).cpu().numpy()
    emu = "f64" if precision == ntbc.FP32 else "bf16"
    l_or, dgrid, dlayers, _ = NV.gradients(pb.cfg, pb.grid, pb.layers, pb.tg_oracle, ids, False, 1, emu)
    dflat = synth.flatten_weights(dlayers).astype(np.float64)
    rg, rw = _rel(tr.d_grid.cpu().numpy(), dgrid), _rel(tr.d_w.cpu().numpy(), dflat)
    log(f"naive train step stage 1 precision {precision}: loss gpu {losses[0]:.7g} oracle {l_or:.7g}; "
        f"rel grid {rg:.3g} weights {rw:.3g}")
    # FP32: float32 rounding; BF16 against its emulation: accumulation order (as the NTBC fused path)
    tol = 1e-4 if precision == ntbc.FP32 else 2e-2
    assert abs(losses[0] - l_or) <= tol * l_or
    assert rg <= tol and rw <= tol


@pytest.mark.parametrize("precision", [ntbc.FP32, ntbc.BF16])
def test_train_step_stage2_updates_only_endpoint_rows(precision):
    pb = _problem("mid", 9)
    cfg = pb.cfg
    ids, ids_d = pb.ids(8, 2048)
    total = 10
    tr = ntbc.Trainer(pb.desc, pb.grid_d, pb.flat_d, pb.tg_gpu, 2048, total, precision=precision, stage2_from=1)
    tr.step(ids_d, 0)                                     # stage 1: everything moves
    g1, w1 = tr.grid.clone(), tr.weights.clone()
    m1, v1, mg1 = tr.m_w.clone(), tr.v_w.clone(), tr.m_grid.clone()
    assert not torch.equal(g1, pb.grid_d) and not torch.equal(w1, pb.flat_d)
    tr.step(ids_d, 1)                                     # stage 2
    assert tr.status() == ntbc.OK
    E = NV.NaiveLayout(cfg.formats).E
    last_in, _ = cfg.layer_dims()[-1]
    off_w = sum(i * o + o for i, o in cfg.layer_dims()[:-1])
    off_b = off_w + last_in * cfg.head_dim
    train = np.zeros(cfg.n_weights, dtype=bool)
    train[off_w:off_w + E * last_in] = True
    train[off_b:off_b + E] = True
    w2, m2, v2 = (t.cpu().numpy() for t in (tr.weights, tr.m_w, tr.v_w))
    w1n, m1n, v1n = (t.cpu().numpy() for t in (w1, m1, v1))
    assert torch.equal(tr.grid, g1) and torch.equal(tr.m_grid, mg1)
    assert np.array_equal(w2[~train], w1n[~train])
    assert np.array_equal(m2[~train], m1n[~train]) and np.array_equal(v2[~train], v1n[~train])
    assert (w2[train] != w1n[train]).mean() > 0.5
    # the trained rows: Adam of step 2 from the GPU's own moments and this step's GPU gradient
    g = tr.d_w.cpu().numpy().astype(np.float64)[train]
    lr = ON.learning_rate(1, 0.005, total)
    p_or, m_or, v_or = ON.adam(w1n[train].astype(np.float64), g, m1n[train].astype(np.float64),
                               v1n[train].astype(np.float64), 2, lr)
    step_err = np.abs(w2[train] - p_or).max() / lr
    log(f"naive stage 2 precision {precision}: trained {train.sum()} values, max |dp - dp_oracle| / lr {step_err:.3g}")
    assert step_err <= 1e-3
    # and the GPU's stage-2 gradient of those rows against the oracle's at the step-2 parameters
    layers = synth.unflatten_weights(cfg, w1n)
    emu = "f64" if precision == ntbc.FP32 else "bf16"
    _, _, dlayers, _ = NV.gradients(cfg, g1.cpu().numpy(), layers, pb.tg_oracle, ids, False, 2, emu)
    dflat = synth.flatten_weights(dlayers).astype(np.float64)
    rw = _rel(g, dflat[train])
    log(f"naive stage 2 precision {precision}: rel endpoint-row gradient {rw:.3g}")
    assert rw <= (1e-4 if precision == ntbc.FP32 else 2e-2)


def test_two_stage_training_learns():
    # 400 steps of the 256^2 five-texture material: stage 1 lowers the loss, stage 2 (the last 20%)
    # keeps it finite, and the trained model decodes better than its initial parameters
    from paper_2407_09543_amd import encode
    pb = _problem("mid", 11)
    tex = [torch.from_numpy(t.texels).cuda() for t in pb.mat.textures]
    model0 = ntbc.Model(pb.desc, pb.flat_d, pb.grid_d)
    words0 = model0.infer(ntbc.FP32)
    total = 400
    tr = ntbc.Trainer(pb.desc, pb.grid_d, pb.flat_d, pb.tg_gpu, 2048, total, precision=ntbc.BF16)
    first = last = None
    for s in range(total):
        ids_d = ntbc.batch_ids(3, s, 2048, pb.cfg.n_positions)
        l = float(tr.step(ids_d, s)[0])
        first = l if s == 0 else first
        last = l
    model = ntbc.Model(pb.desc, tr.weights, tr.grid)
    words = model.infer(ntbc.FP32)
    p0 = encode.psnr_of_words(words0, tex, pb.cfg.formats, 256)
    p1 = encode.psnr_of_words(words, tex, pb.cfg.formats, 256)
    fmt = lambda ps: [None if v is None else round(v, 2) for v in ps]
    log(f"naive 400 steps: loss {first:.4g} -> {last:.4g}; psnr untrained {fmt(p0)} trained {fmt(p1)}")
    assert np.isfinite(last) and last < 0.5 * first
    assert all(b > a for a, b in zip(p0, p1) if a is not None and b is not None)
