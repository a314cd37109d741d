"""GPU parity: operator build and sigma product through the C ABI vs the oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import hbar as ohbar
from oracle import sigma as osig

pytestmark = pytest.mark.gpu

SHAPES = [(2, 1, 3), (3, 2, 4), (5, 7, 11), (10, 20, 0), (13, 37, 2), (17, 45, 9)]


def _cases():
    return [pytest.param(o, v, s, id=f"o{o}v{v}s{s}") for (o, v, s) in SHAPES]


@pytest.mark.parametrize("o,v,seed", _cases())
def test_hbar_blocks(gpu_ctx, o, v, seed):
    print(f"[hbar_blocks o={o} v={v} seed={seed}]", flush=True)
    prob = synth.make_problem(o, v, seed)
    # stronger T1 than the default so every T1 term matters
    prob.t1 = synth.normal(seed, 9, o * v, 0.1).reshape(o, v)
    hb = ohbar.build_hbar_from_problem(prob)
    gpu_ctx.build_from_problem(prob)
    for name in ("Foo", "Fov", "Fvv", "Woooo", "Wooov", "Wovvo", "Wovoo"):
        got = gpu_ctx.export(name).cpu().numpy()
        ref = getattr(hb, name)
        err = np.abs(got - ref).max()
        assert err <= 1e-13 * max(1.0, np.abs(ref).max()), (name, err)
    diag = gpu_ctx.export("diag").cpu().numpy()
    assert np.abs(diag - osig.diagonal(hb)).max() <= 1e-12 * np.abs(diag).max()


@pytest.mark.parametrize("o,v,seed", _cases())
# 64 right-hand sides = 128 real columns: the column-block variant of the ovvo kernel
@pytest.mark.parametrize("nrhs", [1, 3, 64, 70])
@pytest.mark.parametrize("transpose", [False, True])
def test_sigma_fp64(gpu_ctx, o, v, seed, nrhs, transpose):
    print(f"[sigma o={o} v={v} seed={seed} nrhs={nrhs} T={transpose}]", flush=True)
    prob = synth.make_problem(o, v, seed)
    prob.t1 = synth.normal(seed, 9, o * v, 0.1).reshape(o, v)
    hb = ohbar.build_hbar_from_problem(prob)
    gpu_ctx.build_from_problem(prob)
    D = osig.dim(o, v)
    rng = np.random.default_rng(seed + 100 * nrhs)
    x = rng.standard_normal((nrhs, D)) + 1j * rng.standard_normal((nrhs, D))
    y = gpu_ctx.sigma_apply(torch.from_numpy(x).cuda(), transpose=transpose).cpu().numpy()
    ref = osig.sigma_t(hb, x) if transpose else osig.sigma(hb, x)
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err < 1e-13, err


# Wide blocks (1024 and 1030 complex right-hand sides, 2048 and 2060 columns; 160 right-hand
# sides, 320 columns), with the tuner off so that the forward products take the ovvo kernel
# and the unfused linear route: o v = 260 = 2 x 128 + 4 and 264 = 2 x 128 + 8 put the last
# rows of the ovvo contraction on the vector tail kernel instead of a nearly empty last
# 128-row tile (the benzene shape's 7812 = 61 x 128 + 4), its segments m split over 5 to 13
# workgroup layers added in order (at 320 columns some layers hold only the skipped m = j);
# o v = 265 leaves 9 rows, one more than the tail kernel takes, and 64 right-hand sides are
# below the width it needs. o = 13 and 16 (78 and 120 pairs) give the Woo product enough tiles
# for the pipelined kernel, whose epilogue then adds the antisymmetrised ovvo term (no
# separate pass). 1024, 160 and 64 right-hand sides use the column-block loader, 1030 the
# general one.
@pytest.mark.parametrize("o,v,seed", [(13, 20, 5), (11, 24, 6), (5, 53, 7), (16, 30, 8)])
@pytest.mark.parametrize("nrhs", [1024, 1030, 160, 64])
@pytest.mark.parametrize("transpose", [False, True])
def test_sigma_wide_blocks(gpu_ctx, o, v, seed, nrhs, transpose):
    print(f"[sigma wide blocks o={o} v={v} nrhs={nrhs} T={transpose}]", flush=True)
    prob = synth.make_problem(o, v, seed)
    prob.t1 = synth.normal(seed, 9, o * v, 0.1).reshape(o, v)
    hb = ohbar.build_hbar_from_problem(prob)
    D = osig.dim(o, v)
    rng = np.random.default_rng(seed + 100 * nrhs)
    x = rng.standard_normal((nrhs, D)) + 1j * rng.standard_normal((nrhs, D))
    ref = osig.sigma_t(hb, x) if transpose else osig.sigma(hb, x)
    try:
        gpu_ctx.autotune(0)
        gpu_ctx.build_from_problem(prob)
        y = gpu_ctx.sigma_apply(torch.from_numpy(x).cuda(), transpose=transpose).cpu().numpy()
    finally:
        gpu_ctx.autotune(1)
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err < 1e-13, err
    # the entries that take the tail rows' terms: the rows (i, a) = (o - 1, a >= v - t) of the
    # contraction enter sigma at the pairs (j, o - 1), with the same virtual a (the packed
    # 2h1p entry of pair (j, l) and a sits at o + pair(j, l) v + a), relative to their own size
    t = min((o * v) % 128, 8)
    idx = [o + (j * o - j * (j + 1) // 2 + (o - 2 - j)) * v + a
           for j in range(o - 1) for a in range(v - t, v)]
    err_tail = np.abs(y[:, idx] - ref[:, idx]).max() / np.abs(ref[:, idx]).max()
    assert err_tail < 1e-12, err_tail


# FP32 and FP32 + two-term bf16 three-body: a few float32 roundings of the largest terms
# (measured 2e-7 against FP64). BF16_PAIRS: every large contraction carries about 16 bits, and
# sums over o v terms grow that by their cancellation (the oracle's emulation is 8e-6 off FP64
# at this shape), so 5e-5 against FP64 and 4e-5 against the emulation, which rounds the
# Fvv, Foo and Wovvo blocks one by one where the kernel rounds their sum.
@pytest.mark.parametrize("prec,tol,tol_emu", [(1, 2e-6, 2e-6), (2, 2e-6, 2e-6), (3, 5e-5, 4e-5)])
@pytest.mark.parametrize("nrhs", [5, 64, 128])
def test_sigma_reduced_precision(gpu_ctx, prec, tol, tol_emu, nrhs):
    o, v, seed = 13, 37, 2
    print(f"[sigma_mixed prec={prec} nrhs={nrhs}]", flush=True)
    prob = synth.make_problem(o, v, seed)
    hb = ohbar.build_hbar_from_problem(prob)
    from paper_1902_06016_amd import gfcc
    gpu_ctx.build_from_problem(prob, keep=gfcc.KEEP_FP32)
    D = osig.dim(o, v)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((nrhs, D)) + 1j * rng.standard_normal((nrhs, D))
    y = gpu_ctx.sigma_apply(torch.from_numpy(x).cuda(), precision=prec).cpu().numpy()
    ref = osig.sigma(hb, x)
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err < tol, err
    # the oracle's emulation of the same reduced-precision product (float32 operator, the
    # three-body term from two-term bf16 operands)
    from oracle import mixed as omix
    emu = omix.sigma_reduced(omix.f32_hbar(hb), x, bf16_3body=prec == 2, pairs=prec == 3)
    assert np.abs(y - emu).max() <= tol_emu * np.abs(ref).max()
    if prec == 2:
        # the two-term bf16 three-body term: error within 1e-4 of that term's size
        t9 = osig.sigma_parts(hb, x)["T9"]
        e9 = np.abs(y - ref).max() / np.abs(t9).max()
        assert e9 < 1e-4, e9


def test_sigma_fp32_wide_block_tail_rows(gpu_ctx):
    """The FP32 ovvo contraction on a wide block (1024 right-hand sides) at o v = 260 = 2 x 128
    + 4: its last 4 rows take the float tail kernel. Against FP64 at the FP32 tolerance of the
    reduced-precision test and against the oracle's float32 emulation."""
    o, v, seed, nrhs = 13, 20, 5, 1024
    print(f"[sigma fp32 wide block o={o} v={v} nrhs={nrhs}]", flush=True)
    prob = synth.make_problem(o, v, seed)
    hb = ohbar.build_hbar_from_problem(prob)
    from paper_1902_06016_amd import gfcc
    from oracle import mixed as omix
    D = osig.dim(o, v)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((nrhs, D)) + 1j * rng.standard_normal((nrhs, D))
    try:
        gpu_ctx.autotune(0)
        gpu_ctx.build_from_problem(prob, keep=gfcc.KEEP_FP32)
        y = gpu_ctx.sigma_apply(torch.from_numpy(x).cuda(), precision=gfcc.FP32).cpu().numpy()
    finally:
        gpu_ctx.autotune(1)
    ref = osig.sigma(hb, x)
    assert np.abs(y - ref).max() / np.abs(ref).max() < 2e-6
    emu = omix.sigma_reduced(omix.f32_hbar(hb), x, bf16_3body=False, pairs=False)
    assert np.abs(y - emu).max() <= 2e-6 * np.abs(ref).max()
    # the entries the tail rows feed (pairs (j, o - 1), the last 4 virtuals), at the same bound
    idx = [o + (j * o - j * (j + 1) // 2 + (o - 2 - j)) * v + a
           for j in range(o - 1) for a in range(v - 4, v)]
    assert np.abs(y[:, idx] - ref[:, idx]).max() < 2e-6 * np.abs(ref).max()


@pytest.mark.parametrize("o,v,nrhs", [(5, 130, 64), (3, 64, 128)])
def test_sigma_pairs_skip_and_tiles(gpu_ctx, o, v, nrhs):
    """The two-term bf16 ovvo where whole 64-row slabs lie inside a tile's zero segment m = j
    (v >= 64, skipped), with a ragged last M-tile and several column blocks: against FP64 and
    the oracle's emulation, at the bounds of the reduced-precision test above."""
    print(f"[sigma pairs o={o} v={v} nrhs={nrhs}]", flush=True)
    prob = synth.make_problem(o, v, 4)
    hb = ohbar.build_hbar_from_problem(prob)
    from paper_1902_06016_amd import gfcc
    from oracle import mixed as omix
    gpu_ctx.build_from_problem(prob, keep=gfcc.KEEP_FP32)
    D = osig.dim(o, v)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((nrhs, D)) + 1j * rng.standard_normal((nrhs, D))
    y = gpu_ctx.sigma_apply(torch.from_numpy(x).cuda(), precision=gfcc.BF16_PAIRS).cpu().numpy()
    ref = osig.sigma(hb, x)
    assert np.abs(y - ref).max() <= 5e-5 * np.abs(ref).max()
    emu = omix.sigma_reduced(omix.f32_hbar(hb), x, bf16_3body=False, pairs=True)
    assert np.abs(y - emu).max() <= 4e-5 * np.abs(ref).max()


@pytest.mark.parametrize("transpose", [False, True])
def test_sigma_more_than_one_chunk(gpu_ctx, transpose):
    """sigma_apply works through chunks of 2048 right-hand sides: 2100 vectors (a full chunk
    and a ragged one) against the oracle."""
    print(f"[sigma chunks T={transpose}]", flush=True)
    o, v, seed = 5, 7, 11
    prob = synth.make_problem(o, v, seed)
    hb = ohbar.build_hbar_from_problem(prob)
    gpu_ctx.build_from_problem(prob)
    D = osig.dim(o, v)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((2100, D)) + 1j * rng.standard_normal((2100, D))
    y = gpu_ctx.sigma_apply(torch.from_numpy(x).cuda(), transpose=transpose).cpu().numpy()
    ref = osig.sigma_t(hb, x) if transpose else osig.sigma(hb, x)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
