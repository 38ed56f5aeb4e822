"""Every GEMM tile shape and FFT blocking the autotuner may choose gives the
oracle's results; the autotuner and its cache work through the C ABI."""
import json
import os

import numpy as np
import pytest

import synth_inputs as si
from test_gpu_transforms import _check_all, _say, _shtx, _torch

pytestmark = pytest.mark.gpu

SHAPES = {"fp32": [(128, 128), (64, 128), (128, 64)],
          "fp64": [(64, 64), (32, 64), (64, 32)],
          "bf16x3": [(128, 128), (64, 128)],
          "fp16x3": [(128, 128), (64, 128)]}


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16x3", "fp16x3"])
def test_every_tile_shape_matches_oracle(prec):
    shtx = _shtx()
    N, nlat, F = 159, 320, 70
    plan = shtx.Plan(N, "octahedral", nlat, F, prec)
    nlon = plan.ring_lengths()
    shapes = SHAPES[prec]
    for i, t in enumerate(shapes):
        # the direct-shaped launch takes a different shape from the inverse one
        d = shapes[(i + 1) % len(shapes)]
        cap = (6144, 3072, 2048)[i % 3]
        _say(f"shapes {prec} inv {t} dir {d} fft cap {cap}")
        plan.set_shapes(t, d, cap)
        assert tuple(plan.info.inv_tile) == t and tuple(plan.info.dir_tile) == d
        assert plan.info.fft_cap == cap and plan.info.tuned == 0
        _check_all(plan, N, nlon, 11, range(F), prec)
    plan.close()


def test_set_shapes_rejects_unknown_shapes():
    shtx = _shtx()
    plan = shtx.Plan(63, "octahedral", 128, 3, "fp32")
    with pytest.raises(shtx.ShtxError):
        plan.set_shapes((96, 128), (128, 128), 6144)
    with pytest.raises(shtx.ShtxError):
        plan.set_shapes((128, 128), (128, 128), 0)
    a = _torch().from_numpy(si.spectral_fields(63, 3, range(3))).to(plan.complex_dtype).cuda()
    g = plan.inv(a)  # the plan still works with its previous shapes
    assert _torch().isfinite(g).all()


def test_autotune_and_cache(tmp_path):
    torch, shtx = _torch(), _shtx()
    cache = tmp_path / "tune.jsonl"
    os.environ["SHTX_TUNE_CACHE"] = str(cache)
    try:
        N, nlat, F = 255, 512, 64
        ref = shtx.Plan(N, "octahedral", nlat, F, "fp32")
        tuned = shtx.Plan(N, "octahedral", nlat, F, "fp32", autotune=True)
        info = tuned.info
        _say(f"tuned: inv {tuple(info.inv_tile)} dir {tuple(info.dir_tile)} cap {info.fft_cap} ({info.tuned})")
        assert info.tuned == 1
        assert tuple(info.inv_tile) in SHAPES["fp32"] and tuple(info.dir_tile) in SHAPES["fp32"]
        lines = cache.read_text().strip().splitlines()
        assert len(lines) == 1
        rec = json.loads(lines[0])
        assert rec["inv"] == list(info.inv_tile) and rec["dir"] == list(info.dir_tile)
        assert rec["fft_cap"] == info.fft_cap and "gfx" in rec["key"]
        again = shtx.Plan(N, "octahedral", nlat, F, "fp32", autotune=True)
        assert again.info.tuned == 2
        assert tuple(again.info.inv_tile) == tuple(info.inv_tile) and again.info.fft_cap == info.fft_cap
        # tiles change the summation blocking only through the K tiling of the
        # GEMM, which is the same for every shape: results agree closely
        a = torch.from_numpy(si.spectral_fields(N, 5, range(F))).to(torch.complex64).cuda()
        g0, g1 = ref.inv(a), tuned.inv(a)
        scale = g0.abs().max()
        assert ((g0 - g1).abs().max() / scale).item() < 1e-6
        b0, b1 = ref.dir(g0), tuned.dir(g0)
        assert ((b0 - b1).abs().max() / b0.abs().max()).item() < 1e-6
        assert len(cache.read_text().strip().splitlines()) == 1
    finally:
        del os.environ["SHTX_TUNE_CACHE"]
