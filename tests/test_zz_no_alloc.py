"""ntbc_infer_blocks_noalloc (the allocation-free variant of ntbc_infer_blocks: packed weights in the
library's static per-device scratch) gives the same blocks and heads as ntbc_infer_blocks, on two calls
in a row of which the second has a smaller model and block range (the scratch keeps the first call's
contents, so a stale packed-weight read would show)."""
import numpy as np
import pytest
import torch

from cases import model_inputs
from util import ensure_built, log, u64
from paper_2407_09543_amd import ntbc, synth

pytestmark = pytest.mark.gpu


def _device_model(cfg, flat, g):
    desc = ntbc.desc_from_config(cfg)
    w = torch.from_numpy(flat).cuda()
    if "codes" in g:
        return ntbc.Model(desc, w, torch.from_numpy(g["codes"]).cuda(), torch.from_numpy(g["scale"]).cuda(),
                          torch.from_numpy(g["zero"]).cuda())
    return ntbc.Model(desc, w, torch.from_numpy(g["grid"]).cuda())


@pytest.mark.parametrize("precision", [ntbc.BF16, ntbc.FP32, ntbc.FP16])
def test_noalloc_matches_workspace_entry_point(precision):
    ensure_built()
    assert torch.cuda.is_available()
    # first call: the paper-scale network (64-256x3-162, five textures) over a 1024^2 block grid
    cfg1 = synth.config_paper_scale(1024)
    flat1, _, g1 = model_inputs(cfg1, 21)
    m1 = _device_model(cfg1, flat1, g1)
    log(f"noalloc precision {precision}: call 1, {cfg1.n_positions} positions, hidden {cfg1.hidden}")
    ref_w1, ref_h1 = m1.infer(precision, heads=True)
    got_w1, got_h1 = m1.infer_noalloc(precision, heads=True)
    torch.cuda.synchronize()
    assert torch.equal(got_w1, ref_w1)
    assert torch.equal(got_h1, ref_h1)
    # second call: a smaller model (two textures, width 64) on a ragged sub-range
    cfg2 = synth.config_small(256)
    flat2, _, g2 = model_inputs(cfg2, 22)
    m2 = _device_model(cfg2, flat2, g2)
    first, n = 37, cfg2.n_positions - 100
    log(f"noalloc precision {precision}: call 2, blocks [{first}, {first + n}), hidden {cfg2.hidden}")
    ref_w2, ref_h2 = m2.infer(precision, first, n, heads=True)
    got_w2, got_h2 = m2.infer_noalloc(precision, first, n, heads=True)
    torch.cuda.synchronize()
    assert np.array_equal(u64(got_w2), u64(ref_w2))
    assert torch.equal(got_h2, ref_h2)
    # the caller-provided output variant allocates nothing on either side of the boundary
    out = torch.empty_like(ref_w2)
    m2.infer_noalloc(precision, first, n, out=out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref_w2)
