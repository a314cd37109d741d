"""The GEMM autotuner: its split-K variants give the oracle's sigma whichever it picks, with the
tuner on or off, and its choice table names the skinny products of the sigma."""
import numpy as np
import pytest
import torch

import synth
from oracle import hbar as ohbar
from oracle import sigma as osig
from paper_1902_06016_amd import gfcc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("transpose", [False, True])
def test_sigma_with_and_without_the_tuner(gpu_ctx, transpose):
    print(f"[autotune T={transpose}]", flush=True)
    o, v = 12, 30                      # D = 1992: the skinny products are split-K candidates
    prob = synth.make_problem(o, v, 13)
    hb = ohbar.build_hbar_from_problem(prob)
    gpu_ctx.build_from_problem(prob, keep=gfcc.KEEP_FP64 | gfcc.KEEP_TRANSPOSE)
    D = osig.dim(o, v)
    rng = np.random.default_rng(13)
    x = rng.standard_normal((48, D)) + 1j * rng.standard_normal((48, D))
    xt = torch.from_numpy(x).cuda()
    ref = osig.sigma_t(hb, x) if transpose else osig.sigma(hb, x)
    scale = np.abs(ref).max()
    ys = []
    for on in (True, False, True):
        gpu_ctx.autotune(on)
        y = gpu_ctx.sigma_apply(xt, transpose=transpose).cpu().numpy()
        assert np.abs(y - ref).max() <= 1e-12 * scale
        ys.append(y)
        if on:
            ents = gpu_ctx.autotune_entries()
            assert ents, "no product was tuned"
            for e in ents:
                assert e["elem_bytes"] == 8 and e["K"] * 8 >= 4096 and e["us"] > 0
                assert e["splits"] == 0 or e["us"] <= e["generic_us"]
            if not transpose:
                assert any(e["M"] == o + v and e["K"] == D and not e["transA"] for e in ents)
    assert np.abs(ys[0] - ys[1]).max() <= 1e-13 * scale
    # a fresh tuning may pick another variant; both agree to rounding
    assert np.abs(ys[0] - ys[2]).max() <= 1e-13 * scale
    gpu_ctx.autotune(True)
