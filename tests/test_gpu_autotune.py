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
                assert e["elem_bytes"] == 8 and e["us"] > 0
                if e["kind"] in (0, 1):
                    assert e["K"] * 8 >= 4096 and e["tile"] == (0, 0)
                    assert e["splits"] == 0 or e["us"] <= e["generic_us"]
                else:
                    # a sigma, small or small ovvo product: its route or a segmented tile no
                    # slower than it
                    assert e["kind"] in (20, 21, 22, 23)
                    assert e["tile"] == (0, 0) or e["us"] <= e["generic_us"]
            if not transpose:
                assert any(e["kind"] == 20 and e["M"] == o + v and e["K"] == D for e in ents)
                assert any(e["kind"] == 21 and e["M"] == o * (o - 1) // 2
                           and e["K"] == o + v + o * (o - 1) // 2 for e in ents)
    assert np.abs(ys[0] - ys[1]).max() <= 1e-13 * scale
    # a fresh tuning may pick another variant; both agree to rounding
    assert np.abs(ys[0] - ys[2]).max() <= 1e-13 * scale
    gpu_ctx.autotune(True)


def test_small_build_products_in_every_tuner_mode(gpu_ctx):
    """o=10, v=20: every build product has fewer than 64 tiles of 128 x 128 (K6 is 200^3,
    Woooo 100 x 100 x 400 with a transposed B), so the small-product route is tuned between the
    plain routes and the segmented kernel's tiles and split counts; the sigma's ovvo product is
    small as well (the written-out operand against the ovvo kernel). The blocks and the sigma
    match the oracle with the tuner off, untimed at the most split candidates (mode 2) and
    timed; the table names the small products."""
    print("[autotune small build modes]", flush=True)
    o, v = 10, 20
    prob = synth.make_problem(o, v, 5)
    prob.t1 = synth.normal(5, 9, o * v, 0.1).reshape(o, v)
    hb = ohbar.build_hbar_from_problem(prob)
    D = osig.dim(o, v)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((64, D)) + 1j * rng.standard_normal((64, D))
    ref = osig.sigma(hb, x)
    for mode in (0, 2, 1):
        gpu_ctx.autotune(mode)
        gpu_ctx.build_from_problem(prob)
        for name in ("Foo", "Fvv", "Fov", "Woooo", "Wooov", "Wovvo", "Wovoo"):
            g = gpu_ctx.export(name).cpu().numpy()
            r = getattr(hb, name)
            err = np.abs(g - r).max()
            assert err <= 1e-13 * max(1.0, np.abs(r).max()), (mode, name, err)
        y = gpu_ctx.sigma_apply(torch.from_numpy(x).cuda()).cpu().numpy()
        assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max(), mode
        allents = gpu_ctx.autotune_entries()
        ents = [e for e in allents if e["kind"] == 22]
        ovvo = [e for e in allents if e["kind"] == 23]
        if mode == 0:
            assert not ents and not ovvo
        else:
            assert ents, "no small product was tuned"
            # the sigma's ovvo product (o v = 200 rows, o nc = 1280 columns) is small too
            assert len(ovvo) == 1 and ovvo[0]["M"] == o * v and ovvo[0]["N"] == o * 128
            if mode == 2:
                assert all(e["tile"] != (0, 0) for e in ents + ovvo)
                assert any(e["splits"] > 1 for e in ents)
            else:
                assert all(e["tile"] == (0, 0) or e["us"] <= e["generic_us"]
                           for e in ents + ovvo)
    gpu_ctx.autotune(True)


def test_build_products_in_every_tuner_mode(gpu_ctx):
    """o=24, v=90: the O(o^3 v^3) product K6 (2160^3) has 289 tiles, the class tuned between the
    plain pipelined kernel and 2-6 k ranges; Wovoo and Y5 (85 tiles) are split-K products. The
    blocks match the oracle with the tuner off (plain kernels), untimed at the most split
    variants (mode 2) and timed."""
    print("[autotune build modes]", flush=True)
    o, v = 24, 90
    prob = synth.make_problem(o, v, 21)
    prob.t1 = synth.normal(21, 9, o * v, 0.1).reshape(o, v)
    hb = ohbar.build_hbar_from_problem(prob)
    blocks = {}
    for mode in (0, 2, 1):
        gpu_ctx.autotune(mode)
        gpu_ctx.build_from_problem(prob)
        got = {n: gpu_ctx.export(n).cpu().numpy() for n in ("Foo", "Fvv", "Woooo", "Wovvo",
                                                             "Wovoo")}
        for name, g in got.items():
            ref = getattr(hb, name)
            err = np.abs(g - ref).max()
            assert err <= 1e-13 * max(1.0, np.abs(ref).max()), (mode, name, err)
        if mode == 2:
            ents = gpu_ctx.autotune_entries()
            k6 = [e for e in ents if e["M"] == e["N"] == e["K"] == o * v]
            assert k6 and k6[0]["splits"] > 1
            assert any(e["splits"] > 1 and e["M"] == o * v and e["N"] == o * o for e in ents)
        blocks[mode] = got
    for name in blocks[0]:
        scale = np.abs(blocks[0][name]).max()
        assert np.abs(blocks[2][name] - blocks[0][name]).max() <= 1e-13 * max(1.0, scale)
    gpu_ctx.autotune(True)


@pytest.mark.parametrize("o,v,nrhs", [(12, 30, 48), (7, 19, 5), (10, 20, 40)])
def test_every_fused_sigma_variant(gpu_ctx, o, v, nrhs):
    """The forward sigma with its two fused products pinned to each tile shape and split count
    (and to the unfused route) matches the oracle: ragged tiles in M (P pairs, o + v rows), in
    N (2 nrhs columns) and in every K segment (o, v, P)."""
    print(f"[fused sigma variants o={o} v={v} nrhs={nrhs}]", flush=True)
    prob = synth.make_problem(o, v, 31)
    hb = ohbar.build_hbar_from_problem(prob)
    gpu_ctx.build_from_problem(prob)
    D = osig.dim(o, v)
    rng = np.random.default_rng(31)
    x = rng.standard_normal((nrhs, D)) + 1j * rng.standard_normal((nrhs, D))
    xt = torch.from_numpy(x).cuda()
    ref = osig.sigma(hb, x)
    scale = np.abs(ref).max()
    variants = [(0, 0, 1)] + [(tm, tn, sp) for tm in (32, 64, 128) for tn in (64, 128)
                              for sp in (1, 3)]
    try:
        for tm, tn, sp in variants:
            gpu_ctx.autotune(True)
            gpu_ctx.autotune_pin(20, tm, tn, sp)
            gpu_ctx.autotune_pin(21, tm, tn, sp)
            y = gpu_ctx.sigma_apply(xt).cpu().numpy()
            err = np.abs(y - ref).max()
            assert err <= 1e-12 * scale, (tm, tn, sp, err / scale)
        with pytest.raises(gfcc.GfccError):
            gpu_ctx.autotune_pin(21, 48, 64, 1)
        with pytest.raises(gfcc.GfccError):
            gpu_ctx.autotune_pin(5, 32, 64, 1)
    finally:
        gpu_ctx.autotune(True)
