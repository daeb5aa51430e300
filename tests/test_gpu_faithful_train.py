"""GPU parity of the paper layout's training step (ntbc_faithful_train_step: endpoint network + per-texel
colour network, SELU, FP32 products; Sec. 3.2, Sec. 3.4, Sec. 4.1) against its oracle
(oracle.faithful.gradients / train_step).

* Gradients of both networks and both grids, and the losses, at the initial parameters, without and
  with QAT, with the atomic and the fixed-point (deterministic) grid scatter, with a colour grid whose
  finest level matches the texel grid (per-block texel sums) and one finer than it (the generic
  scatter): within float32 rounding of the FP64 oracle (relative norm 1e-4, measured about 1e-6;
  losses 1e-5).  Blocks where
  a texel's two nearest palette entries are within 1e-6 of each other are left out of the batch: there
  the float32 and float64 argmax of the decoded-colour terms may differ (a different straight-through
  target, not a rounding difference).
* The first Adam step: every parameter with a gradient moves by lr g / (|g| + eps) of its set's learning
  rate (grids lr_grid, networks lr_mlp, the warm-up's first step), the others stay; the moments are
  (1 - beta) g and (1 - beta2) g^2.
* Deterministic steps repeat bitwise.
* Training learns in both material layouts: the loss falls and the trained models' blocks (decoded by
  ntbc_faithful_infer from the FP32 grids) beat the untrained ones in PSNR; after QAT in the last 10%
  of the steps, the grids quantised to 8 bits (ntbc_quantize_grid) decode within 0.5 dB of the FP32
  master grids."""
import numpy as np
import pytest
import torch

from cases import near_tie_positions
from util import ensure_built, log
from oracle import bc as OB
from oracle import faithful as F
from oracle import ntbc as ON
from oracle.ntbc import BC1, BC4
from paper_2407_09543_amd import encode, ntbc, synth

pytestmark = pytest.mark.gpu

SIZE = 128                                             # 32 x 32 blocks, 128 x 128 texels
EP = dict(n_levels=3, base_res=4, n_features=2)        # 4 .. 16 over the block grid
# 8 .. 128 over the texel grid: levels 8 .. 64 fit the LDS pre-sum of the grid scatter, level 128 takes
# the per-block texel sums; COL_FINE adds a level finer than the texel grid (256: the generic scatter)
COL = dict(n_levels=5, base_res=8, n_features=2)
COL_FINE = dict(n_levels=6, base_res=8, n_features=2)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    assert torch.cuda.is_available()


class Problem:
    """The 128^2 BC1 + BC4 material, the textures of one model, targets on both sides, parameters."""

    def __init__(self, which, seed, col=COL):
        self.col = col
        mat = synth.material_small(SIZE, seed)
        texs = [t for t in mat.textures if which == "all" or (t.fmt == BC1) == (which == "bc1")]
        self.formats = [t.fmt for t in texs]
        blocks = [OB.image_to_blocks(t.texels) for t in texs]
        ref = [OB.bc1_encode_ref(b) if t.fmt == BC1 else OB.bc4_encode_ref(b[..., 0]) for b, t in zip(blocks, texs)]
        self.tg_oracle = ON.Targets(self.formats, ref, blocks)
        self.tex = [torch.from_numpy(t.texels).cuda() for t in texs]
        self.tg_gpu = ntbc.Targets(torch.stack([ntbc.encode_ref(t, f) for t, f in zip(self.tex, self.formats)]),
                                   self.tex)
        rng = np.random.default_rng(seed)
        e, c = F.output_nodes(self.formats)
        self.ew, self.cw = self._net(rng, 2 * EP["n_levels"], e), self._net(rng, 2 * col["n_levels"], c)
        self.eg = rng.uniform(-0.5, 0.5, (F.grid_vertices(EP), 2)).astype(np.float32)
        self.cg = rng.uniform(-0.5, 0.5, (F.grid_vertices(col), 2)).astype(np.float32)
        self.bw = self.bh = SIZE // 4

    @staticmethod
    def _net(rng, n_in, n_out):
        return [((rng.standard_normal((o, i)) * np.sqrt(1.0 / i)).astype(np.float32),
                 (0.1 * rng.standard_normal(o)).astype(np.float32)) for i, o in F.layer_dims(n_in, n_out)]

    @staticmethod
    def flat(layers):
        return np.concatenate([np.concatenate([w.ravel(), b]) for w, b in layers]).astype(np.float32)

    def trainer(self, batch, total, **kw):
        t = lambda a: torch.from_numpy(a).cuda()
        return ntbc.FaithfulTrainer(self.formats, self.bw, self.bh, t(self.eg), t(self.cg), t(self.flat(self.ew)),
                                    t(self.flat(self.cw)), self.tg_gpu, batch, total, ep_levels=EP["n_levels"],
                                    ep_base_res=EP["base_res"], col_levels=self.col["n_levels"],
                                    col_base_res=self.col["base_res"], **kw)

    def oracle(self, ids, qat):
        return F.gradients(self.formats, self.eg, self.ew, self.cg, self.cw, self.tg_oracle, ids, self.bw, self.bh,
                           qat, ep_cfg=EP, col_cfg=self.col)

    def clean_ids(self, seed, n, qat):
        """n distinct block ids without near ties of the decoded-colour argmax (oracle heads)."""
        ids = np.random.default_rng(seed).choice(self.bw * self.bh, min(2 * n, self.bw * self.bh), replace=False)
        y = self.oracle(ids, qat)[5]
        keep = ids[~near_tie_positions(self, y, ids)][:n]
        assert len(keep) == n
        return keep.astype(np.int32)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("qat,col,det", [(False, COL, False), (True, COL, False), (False, COL_FINE, False),
                                         (True, COL, True)])
@pytest.mark.parametrize("which", ["all", "bc1", "bc4"])
def test_gradients_match_oracle(which, qat, col, det):
    # "all": the aggressive layout's one model over both textures; "bc1" / "bc4": the conservative
    # layout's two models; det: the fixed-point grid scatter
    pb = Problem(which, 3, col)
    ids = pb.clean_ids(4, 512, qat)
    tr = pb.trainer(len(ids), 100, deterministic=det)
    losses = tr.step(torch.from_numpy(ids).cuda(), 0, qat=qat).cpu().numpy()
    l_or, dge, dle, dgc, dlc, _ = pb.oracle(ids, qat)
    rel = [_rel(tr.d_ep_grid.cpu().numpy(), dge), _rel(tr.d_col_grid.cpu().numpy(), dgc),
           _rel(tr.d_ep_weights.cpu().numpy(), Problem.flat(dle).astype(np.float64)),
           _rel(tr.d_col_weights.cpu().numpy(), Problem.flat(dlc).astype(np.float64))]
    log(f"paper layout training {which} qat={qat} colour levels {col['n_levels']} det={det}: losses gpu "
        f"{losses[:4]} oracle {l_or}; rel grad ep grid {rel[0]:.3g} col grid {rel[1]:.3g} ep weights {rel[2]:.3g} "
        f"col weights {rel[3]:.3g}")
    assert losses[4] == 0
    assert np.allclose(losses[:4], l_or, rtol=1e-5, atol=1e-9)
    assert max(rel) <= 1e-4


def test_first_adam_step():
    pb = Problem("all", 5)
    ids = torch.from_numpy(pb.clean_ids(6, 256, False)).cuda()
    tr = pb.trainer(256, 50, lr_grid=0.01, lr_mlp=0.005)
    before = [t.cpu().numpy().copy() for t in tr.params]
    tr.step(ids, 0)
    torch.cuda.synchronize()
    b1, b2 = np.float32(0.9), np.float32(0.999)
    for k, lr in enumerate((0.001, 0.001, 0.0005, 0.0005)):   # warm-up step 1 of 10
        g = tr.grads[k].cpu().numpy().astype(np.float64)
        p0, p1 = before[k].astype(np.float64), tr.params[k].cpu().numpy().astype(np.float64)
        m1, v1 = tr.m[k].cpu().numpy(), tr.v[k].cpu().numpy()
        moved = g != 0
        assert moved.mean() > 0.05
        assert (p1[~moved] == p0[~moved]).all()
        step = p1[moved] - p0[moved]
        want = -lr * g[moved] / (np.abs(g[moved]) + 1e-15)
        err = np.abs(step - want) - 2.0 ** -23 * np.abs(p0[moved])
        log(f"  set {k}: {moved.sum()} moved, max |step - lr sign(-g)| beyond a rounding of p: {err.max():.3g}")
        assert (err <= 1e-4 * lr).all()
        assert np.allclose(m1, (1 - b1) * g, rtol=2.0 ** -21, atol=0)
        assert np.allclose(v1, (1 - b2) * g * g, rtol=2.0 ** -20, atol=0)


def test_deterministic_steps_repeat_bitwise():
    pb = Problem("all", 4)
    ids = torch.from_numpy(pb.clean_ids(5, 512, False)).cuda()
    runs = []
    for _ in range(2):
        tr = pb.trainer(512, 20, deterministic=True)
        for s in range(3):
            tr.step(ids, s)
        runs.append([t.clone() for t in tr.params + tr.grads])
    assert all(torch.equal(a, b) for a, b in zip(*runs))


def _grid_desc(g):
    """A model description whose grid has the shape of g (for ntbc_quantize_grid)."""
    d = ntbc.ModelDesc()
    d.n_levels, d.base_res, d.n_features, d.grid_dtype = g["n_levels"], g["base_res"], 2, ntbc.GRID_F32
    d.hidden_width, d.n_hidden, d.n_textures, d.blocks_w, d.blocks_h = 64, 1, 1, 1, 1
    d.formats[0] = BC1
    return d


def _infer_words(pb, formats, tr, u8=False):
    grids = [tr.ep_grid, tr.col_grid]
    q = [{}, {}]
    if u8:
        # the deployed model: both grids quantised to 8 bits per level (Sec. 3.3)
        for k, g in enumerate((EP, pb.col)):
            codes, scale, zero = ntbc.quantize_grid(_grid_desc(g), grids[k])
            grids[k] = codes
            q[k] = {"scale": scale, "zero": zero}
    m = ntbc.FaithfulModel(formats, pb.bw, pb.bh, grids[0], grids[1], tr.ep_weights, tr.col_weights,
                           ep_levels=EP["n_levels"], ep_base_res=EP["base_res"], col_levels=pb.col["n_levels"],
                           col_base_res=pb.col["base_res"], ep_scale=q[0].get("scale"), ep_zero=q[0].get("zero"),
                           col_scale=q[1].get("scale"), col_zero=q[1].get("zero"))
    return m.infer()


@pytest.mark.parametrize("layout", ["aggressive", "conservative"])
def test_training_learns(layout):
    groups = ["all"] if layout == "aggressive" else ["bc1", "bc4"]
    total, batch = 300, 512
    for which in groups:
        pb = Problem(which, 7)
        tr = pb.trainer(batch, total)
        words0 = _infer_words(pb, pb.formats, tr)
        first = last = None
        for s in range(total):
            ids = ntbc.batch_ids(8, s, batch, pb.bw * pb.bh)
            l = tr.step(ids, s, qat=s >= total - total // 10).cpu().numpy()   # the last 10% with QAT
            assert l[4] == 0
            first = l[:4].sum() if s == 0 else first
            last = l[:4].sum()
        words = _infer_words(pb, pb.formats, tr)
        words8 = _infer_words(pb, pb.formats, tr, u8=True)
        p0 = encode.psnr_of_words(words0, pb.tex, pb.formats, SIZE)
        p1 = encode.psnr_of_words(words, pb.tex, pb.formats, SIZE)
        p8 = encode.psnr_of_words(words8, pb.tex, pb.formats, SIZE)
        log(f"paper layout {layout} model {which}: loss {first:.4g} -> {last:.4g}; psnr {np.round(p0, 2).tolist()} -> "
            f"{np.round(p1, 2).tolist()} (FP32 grids), {np.round(p8, 2).tolist()} (8-bit grids)")
        assert last < 0.5 * first
        assert all(b > a + 3.0 for a, b in zip(p0, p1))
        # trained with QAT at the end, the 8-bit grids decode about as well as the FP32 master grids
        assert all(abs(b - a) < 0.5 for a, b in zip(p1, p8))


def test_rejects():
    pb = Problem("all", 9)
    tr = pb.trainer(64, 10)
    ids = torch.zeros(64, dtype=torch.int32, device="cuda")
    tr.h.precision = ntbc.BF16
    with pytest.raises(ntbc.NtbcError) as e:
        tr.step(ids, 0)
    assert e.value.status == ntbc.EUNSUPPORTED
    tr.h.precision = ntbc.FP32
    tr.desc.grid_dtype = ntbc.GRID_U8
    with pytest.raises(ntbc.NtbcError):
        tr.step(ids, 0)
    tr.desc.grid_dtype = ntbc.GRID_F32
    with pytest.raises(ntbc.NtbcError):                  # the workspace was sized for 64 blocks
        tr.step(torch.zeros(65, dtype=torch.int32, device="cuda"), 0)
    tr.step(ids, 0)                                      # and the step itself still runs
    assert tr.losses.cpu().numpy()[4] == 0
