"""GPU encode pipeline: device batch ids equal the host generator; a trained network beats the
untrained one; the per-block judge never makes a block worse than the better of NTBC and reference."""
import numpy as np
import pytest
import torch

from util import ensure_built, log, u64
from oracle import bc as OB
from paper_2407_09543_amd import encode, ntbc, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    assert torch.cuda.is_available()


def test_device_batch_ids_match_host_generator():
    for seed, step, batch, n in ((1, 0, 512, 4096), (3, 19999, 65536, 1 << 20), (7, 5, 1000, 77)):
        got = ntbc.batch_ids(seed, step, batch, n).cpu().numpy()
        assert np.array_equal(got, synth.batch_ids(seed, step, batch, n))


def test_trained_network_beats_untrained_and_judge():
    cfg = synth.config_mid(256)
    mat = synth.material_five(256, 4)
    tex = [torch.from_numpy(t.texels).cuda() for t in mat.textures]
    res = encode.encode_material(tex, cfg, steps=600, batch=2048, seed=4, kappa=1.0, delta=0.0, log_every=100)
    trained = encode.psnr_of_words(res.ntbc_words, tex, cfg.formats, 256)
    ref = encode.psnr_of_words(res.ref_words, tex, cfg.formats, 256)
    judged = encode.psnr_of_words(res.words, tex, cfg.formats, 256)
    # the same pipeline with the untrained initial parameters
    desc = ntbc.desc_from_config(cfg)
    codes, scale, zero = ntbc.quantize_grid(desc, torch.from_numpy(synth.init_grid(cfg, 4)).cuda())
    w0 = torch.from_numpy(synth.flatten_weights(synth.init_weights(cfg, 4))).cuda()
    untrained = encode.psnr_of_words(ntbc.Model(desc, w0, codes, scale, zero).infer(ntbc.BF16), tex, cfg.formats, 256)
    log(f"psnr trained {np.round(trained, 2)} untrained {np.round(untrained, 2)} ref {np.round(ref, 2)} "
        f"judged {np.round(judged, 2)} fallback {res.fallback_blocks} losses {res.losses[-1]}")
    assert all(t > u + 5.0 for t, u in zip(trained, untrained))
    # kappa = 1, delta = 0: every block is the better of the two, so the judged texture is at least
    # as good as both
    assert all(j >= max(t, r) - 1e-9 for j, t, r in zip(judged, trained, ref))
    for t in range(len(cfg.formats)):
        words, n_w, r_w = u64(res.words[t]), u64(res.ntbc_words[t]), u64(res.ref_words[t])
        assert ((words == n_w) | (words == r_w)).all()
        assert int((words != n_w).sum()) <= res.fallback_blocks[t]
