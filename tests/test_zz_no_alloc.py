"""The allocation-free inverse transform (shtx_inv_trans_noalloc) against
shtx_inv_trans, through the C ABI: the same kernels on the same inputs, so
the outputs must be bit-identical.  Two calls in a row share the static
scratch, the second with a smaller input, in the single-precision, split-half
and double-precision forms; a plan whose workspace exceeds the static array is
refused before anything runs."""
import ctypes

import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu


def _env():
    import torch
    import paper_1908_06097_amd as shtx
    if not torch.cuda.is_available():
        pytest.fail("GPU test without a GPU")
    return torch, shtx


def _noalloc(torch, lib, plan, spec, out):
    stream = torch.cuda.current_stream().cuda_stream
    return lib.shtx_inv_trans_noalloc(plan._h, ctypes.c_void_p(spec.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                      ctypes.c_void_p(stream))


@pytest.mark.parametrize("prec", ["fp32", "fp16x3", "fp64"])
def test_noalloc_matches_inv_trans_twice(prec):
    torch, shtx = _env()
    lib = shtx.load_library()
    # the second call is smaller: fewer fields and a lower truncation
    for N, nlat, F in ((159, 320, 70), (63, 128, 5)):
        print(f"noalloc {prec} T{N} O{nlat // 2} F={F}", flush=True)
        plan = shtx.Plan(N, "octahedral", nlat, F, prec)
        spec = torch.from_numpy(si.spectral_fields(N, 41, range(F))).to(plan.complex_dtype).cuda()
        ref = plan.inv(spec)
        out = torch.full_like(ref, float("nan"))
        assert _noalloc(torch, lib, plan, spec, out) == 0
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        plan.close()


def test_noalloc_refuses_oversized_workspace():
    torch, shtx = _env()
    lib = shtx.load_library()
    # T255 on O256 with 411 fields: 411 x 100568 complex64 = 331 MB > 256 MiB
    plan = shtx.Plan(255, "octahedral", 512, 411, "fp32")
    assert plan.info.nfour * plan.nfld * 8 > (256 << 20)
    spec = torch.zeros((plan.nfld, plan.nspec), dtype=plan.complex_dtype, device="cuda")
    out = torch.full((plan.nfld, plan.npts), 7.0, dtype=plan.real_dtype, device="cuda")
    assert _noalloc(torch, lib, plan, spec, out) == -5
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())  # nothing was launched
    assert lib.shtx_strerror(-5).decode().startswith("transform needs more scratch")
    plan.close()
