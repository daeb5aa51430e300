"""GPU parity of the optimiser step and of mid-run gradients (Sec. 3.4: Adam with beta 0.9/0.999,
eps 1e-15, learning rates 0.01 and 0.005, warm-up then cosine annealing; Sec. 3.3: QAT in the extra
steps).

* Adam: after each ntbc_train_step the parameters and both moments equal the oracle's Adam update
  (oracle.ntbc.adam with the oracle's learning_rate) applied to the state before the step and the
  gradient the step computed (d_grid, d_weights), element by element, at steps 0-11 (both sides of the
  warm-up boundary at step 10) and at the last step of the schedule.
* Mid-run gradients: the 1024^2 five-texture model (48-128x3-162, six FP32 grid levels 8..256) trained
  on the GPU for 2,000 + 200 QAT steps at batch 16,384; at step 1,000 (no QAT) and after step 2,200
  (QAT on) the GPU's end-to-end gradients (forward, loss with the straight-through estimator, backward)
  equal the oracle's at the same parameters."""
import dataclasses

import numpy as np
import pytest
import torch

from cases import TrainProblem, near_tie_positions
from util import ensure_built, log
from oracle import grid as OG
from oracle import mlp as OMLP
from oracle import ntbc as ON
from paper_2407_09543_amd import ntbc, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    assert torch.cuda.is_available()


def F32(x):
    return float(np.float32(x))


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _check_adam(name, p0, g, m0, v0, p1, m1, v1, t, lr):
    """GPU (p1, m1, v1) against the oracle's Adam update of (p0, m0, v0) with gradient g.  The GPU keeps
    FP32 state: each moment is within a few float32 roundings of its two terms (which may cancel, so
    the bound is relative to the terms, not to the result), and the parameter within a float32 rounding
    of itself plus the update's error through the moments."""
    b1, b2, eps = F32(0.9), F32(0.999), F32(1e-15)
    # the hyper-parameters cross the C ABI as float32 (ntbc_hparams): the oracle takes the same values
    p_or, m_or, v_or = ON.adam(p0, g, m0, v0, t, lr, b1=b1, b2=b2, eps=eps)
    u = 2.0 ** -22  # four float32 roundings
    tol_m = u * (b1 * np.abs(m0) + (1 - b1) * np.abs(g))
    tol_v = u * (b2 * np.abs(v0) + (1 - b2) * g * g)
    c1, c2 = 1.0 / (1.0 - b1 ** t), 1.0 / (1.0 - b2 ** t)
    den = np.sqrt(np.abs(v_or) * c2) + eps
    step = np.abs(p_or - p0)
    tol_p = u * np.abs(p_or) + 1e-5 * step + lr * c1 * tol_m / den + 0.5 * step * c2 * tol_v / np.maximum(
        np.abs(v_or) * c2, 1e-300)
    log(f"  {name}: t={t} lr={lr:.6g} max|dp| {np.abs(p1 - p_or).max():.3g} (max step {step.max():.3g}) "
        f"max|dm| {np.abs(m1 - m_or).max():.3g} max|dv| {np.abs(v1 - v_or).max():.3g}")
    assert np.all(np.abs(m1 - m_or) <= tol_m), f"{name}: first moment differs"
    assert np.all(np.abs(v1 - v_or) <= tol_v), f"{name}: second moment differs"
    assert np.all(np.abs(p1 - p_or) <= tol_p), f"{name}: parameter update differs"


def test_adam_updates_elementwise_across_warmup():
    cfg = dataclasses.replace(synth.config_mid(256), grid_u8=False)
    pb = TrainProblem(cfg, synth.material_five(256, 11), 11)
    total = 100
    lr_grid, lr_mlp = 0.01, 0.005
    tr = ntbc.Trainer(pb.desc, pb.grid_d, pb.flat_d, pb.tg_gpu, 1024, total, lr_grid=lr_grid, lr_mlp=lr_mlp)
    for step in list(range(12)) + [total - 1]:
        before = [_np(x) for x in (tr.grid, tr.m_grid, tr.v_grid, tr.weights, tr.m_w, tr.v_w)]
        ids = ntbc.batch_ids(11, step, 1024, cfg.n_positions)
        losses = tr.step(ids, step).cpu().numpy()
        assert losses[4] == 0.0
        g_grid, g_w = _np(tr.d_grid), _np(tr.d_w)
        assert np.abs(g_w).max() > 0 and np.abs(g_grid).max() > 0
        log(f"step {step}")
        _check_adam("grid", before[0], g_grid, before[1], before[2], _np(tr.grid), _np(tr.m_grid), _np(tr.v_grid),
                    step + 1, ON.learning_rate(step, F32(lr_grid), total))
        _check_adam("mlp", before[3], g_w, before[4], before[5], _np(tr.weights), _np(tr.m_w), _np(tr.v_w),
                    step + 1, ON.learning_rate(step, F32(lr_mlp), total))
    # the schedule itself: the last warm-up step and the first cosine step both use the full rate
    assert ON.learning_rate(9, 1.0, total) == 1.0 and ON.learning_rate(10, 1.0, total) == 1.0
    assert ON.learning_rate(11, 1.0, total) < 1.0


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_mid_run_gradients_config2_with_qat():
    cfg = dataclasses.replace(synth.config_mid(1024), grid_u8=False)
    mat = synth.material_five(1024, 2)
    pb = TrainProblem(cfg, mat, 2)
    grid0 = synth.init_grid(cfg, 2)
    w0 = synth.flatten_weights(synth.init_weights(cfg, 2))
    base, extra, batch = 2000, 200, 16384
    tr = ntbc.Trainer(pb.desc, torch.from_numpy(grid0).cuda(), torch.from_numpy(w0).cuda(), pb.tg_gpu, batch,
                      base + extra)
    snaps = {}
    ids_d = torch.empty(batch, dtype=torch.int32, device="cuda")
    skipped = torch.zeros((), dtype=torch.float32, device="cuda")
    for s in range(base + extra):
        if s == 1000:
            snaps[1000] = (tr.grid.clone(), tr.weights.clone(), False)
        ntbc.batch_ids(2, s, batch, cfg.n_positions, out=ids_d)
        skipped += tr.step(ids_d, s, qat=s >= base)[4]
    snaps[2200] = (tr.grid.clone(), tr.weights.clone(), True)
    assert float(skipped) == 0.0
    for step, (grid_d, w_d, qat) in snaps.items():
        ids_all = synth.batch_ids(77, step, 2048, cfg.n_positions)
        grid_np = grid_d.cpu().numpy()
        layers = synth.unflatten_weights(cfg, w_d.cpu().numpy().astype(np.float64))
        # a trained model predicts colours close to the texels, and a texel often sits near the middle of
        # two palette entries, so some decisions of the decoded-colour terms (a texel's two nearest
        # entries, or a predicted BC4 endpoint pair: the mode switch) lie within float32 noise of a tie.
        # There the float32 and float64 argmax may differ, and with T = 0.01 one flipped choice moves a
        # whole softmax term.  Positions with a decision gap below 2e-6 (four times the largest head
        # difference seen, 5e-7) are left out and the rest compared tightly
        _, _, _, y0 = ON.gradients(cfg, grid_np, layers, pb.tg_oracle, ids_all, qat=qat)
        keep = ~near_tie_positions(pb, y0, ids_all, gap=2e-6)
        # the same for the ReLU kinks: a hidden pre-activation within float32 noise of zero (the
        # 128-term dot products carry ~1e-6 of it; gap 1e-5) may switch its unit on one side only,
        # which moves that position's whole dX through the unit: leave such positions out as well
        g = OG.fake_quant_grid(grid_np, cfg.n_levels, cfg.base_res)[0] if qat else grid_np.astype(np.float64)
        x = OG.features(OG.split_levels(g, cfg.n_levels, cfg.base_res), ids_all % cfg.blocks_w,
                        ids_all // cfg.blocks_w, cfg.blocks_w, cfg.blocks_h)
        _, (_, zs) = OMLP.forward(layers, x)
        kink = np.zeros(len(ids_all), dtype=bool)
        for z in zs[:-1]:
            kink |= (np.abs(z) < 1e-5).any(axis=1)
        keep &= ~kink
        ids = ids_all[keep]
        ids_t = torch.from_numpy(ids).cuda()
        y = ntbc.forward(pb.desc, grid_d, w_d, ids_t, qat=qat)
        losses, dh = ntbc.loss_grad(pb.desc, pb.tg_gpu, y, ids_t)
        dg, dw = ntbc.backward(pb.desc, grid_d, w_d, ids_t, dh, qat=qat)
        l_or, dgrid, dlayers, y_or = ON.gradients(cfg, grid_np, layers, pb.tg_oracle, ids, qat=qat)
        dflat = synth.flatten_weights(dlayers).astype(np.float64)
        rg, rw = _rel(dg.cpu().numpy(), dgrid), _rel(dw.cpu().numpy(), dflat)
        dy = float(np.abs(y.cpu().numpy() - y_or).max())
        log(f"step {step} qat={qat}: kept {keep.sum()}/{len(keep)} positions ({kink.sum()} at a ReLU kink); losses gpu {losses.cpu().numpy()[:4]} "
            f"oracle {l_or}; max|dY| {dy:.3g}; rel grid {rg:.3g} weights {rw:.3g}")
        assert keep.mean() >= 0.5
        assert dy <= 1e-5
        assert np.allclose(losses.cpu().numpy()[:4], l_or, rtol=1e-4, atol=1e-8)
        assert rg <= 1e-3 and rw <= 1e-3


@pytest.mark.parametrize("precision", [ntbc.FP32, ntbc.BF16])
def test_deterministic_mode(precision):
    # hparams.deterministic = 1: five steps (two with QAT) from the same state give the same bits twice;
    # its grid gradient (64-bit fixed-point sums) agrees with the FP32-atomic one to far below FP32's
    # resolution of the sums: ||difference|| <= 1e-6 ||gradient||.  The FP32 products take the unfused
    # path (unsplit weight products in this mode), the bfloat16 products the fused one.
    cfg = dataclasses.replace(synth.config_mid(256), grid_u8=False)
    pb = TrainProblem(cfg, synth.material_five(256, 12), 12)
    ids = [ntbc.batch_ids(12, s, 2048, cfg.n_positions) for s in range(5)]
    states = []
    for rep in range(2):
        tr = ntbc.Trainer(pb.desc, pb.grid_d, pb.flat_d, pb.tg_gpu, 2048, 5, precision=precision, deterministic=True)
        for s in range(5):
            tr.step(ids[s], s, qat=s >= 3)
        torch.cuda.synchronize()
        states.append([t.clone() for t in (tr.grid, tr.weights, tr.m_grid, tr.v_grid, tr.m_w, tr.v_w, tr.d_grid, tr.d_w)])
    same = [bool(torch.equal(a, b)) for a, b in zip(*states)]
    log(f"deterministic precision {precision}: identical state tensors {same}")
    assert all(same)
    grads = {}
    for det in (False, True):
        tr = ntbc.Trainer(pb.desc, pb.grid_d, pb.flat_d, pb.tg_gpu, 2048, 5, precision=precision, deterministic=det)
        tr.step(ids[0], 0)
        grads[det] = (tr.d_grid.double().cpu(), tr.d_w.double().cpu())
    rg = float((grads[True][0] - grads[False][0]).norm() / grads[False][0].norm())
    rw = float((grads[True][1] - grads[False][1]).norm() / grads[False][1].norm())
    log(f"  atomic vs deterministic: rel grid {rg:.3g} weights {rw:.3g}")
    assert rg <= 1e-6 and rw <= 1e-6


@pytest.mark.parametrize("qat", [False, True])
def test_bf16_train_step_gradients(qat):
    # the gradient that one bfloat16 training step computes (its d_grid and d_weights: forward with the
    # layers chained in registers, loss with the straight-through estimator, backward) against the
    # oracle's at the same parameters with the bfloat16 product emulation.  Positions whose heads the
    # two evaluate differently (a bfloat16 rounding flip somewhere in the network: |dY| > 1e-6) or
    # with a decision near a tie are left out before the step, so both sides see the same decisions
    cfg = dataclasses.replace(synth.config_mid(256), grid_u8=False)
    pb = TrainProblem(cfg, synth.material_five(256, 13), 13)
    cand = synth.batch_ids(13, 0, 3000, cfg.n_positions)
    y = ntbc.forward(pb.desc, pb.grid_d, pb.flat_d, torch.from_numpy(cand).cuda(), qat=qat,
                     precision=ntbc.BF16).cpu().numpy()
    _, _, _, y_or = ON.gradients(cfg, pb.grid, pb.layers, pb.tg_oracle, cand, qat=qat, precision="bf16")
    keep = (np.abs(y - y_or).max(axis=1) <= 1e-6) & ~near_tie_positions(pb, y_or, cand, gap=1e-5)
    ids = cand[keep]
    tr = ntbc.Trainer(pb.desc, pb.grid_d, pb.flat_d, pb.tg_gpu, len(ids), 10, precision=ntbc.BF16)
    losses = tr.step(torch.from_numpy(ids).cuda(), 0, qat=qat).cpu().numpy()
    l_or, dgrid, dlayers, _ = ON.gradients(cfg, pb.grid, pb.layers, pb.tg_oracle, ids, qat=qat, precision="bf16")
    dflat = synth.flatten_weights(dlayers).astype(np.float64)
    rg, rw = _rel(tr.d_grid.cpu().numpy(), dgrid), _rel(tr.d_w.cpu().numpy(), dflat)
    log(f"bf16 train step qat={qat}: kept {keep.sum()}/{len(cand)}; losses gpu {losses[:4]} oracle {l_or}; "
        f"rel grid {rg:.3g} weights {rw:.3g}")
    assert keep.mean() >= 0.5
    assert np.allclose(losses[:4], l_or, rtol=1e-4, atol=1e-9)
    assert rg <= 5e-3 and rw <= 5e-3
