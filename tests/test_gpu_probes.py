"""Peak probes (shtx_probe_peak): the rates bench.py reports beside the
published MI355X peaks.  Plausibility bounds only: each measured rate must lie
between a third of and just above the vendor figure for its unit (the FP32
vector loop uses no packed instructions, so its floor is a third of half the
published 157.3 TFLOP/s)."""
import ctypes

import pytest

pytestmark = pytest.mark.gpu

# (kind, lower, upper) in TFLOP/s or GB/s
BOUNDS = [("mfma_f64", 78.6 / 3, 78.6 * 1.05), ("mfma_f32", 157.3 / 3, 157.3 * 1.05),
          ("mfma_bf16", 2500 / 3, 2500 * 1.05), ("mfma_f16", 2500 / 3, 2500 * 1.05),
          ("valu_f32", 78.6 / 3, 157.3 * 1.05), ("hbm_copy", 8000 / 3, 8000 * 1.05),
          ("hbm_read", 8000 / 3, 8000 * 1.05)]


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test without a GPU")
    return torch


@pytest.mark.parametrize("kind,lo,hi", BOUNDS)
def test_probe_rate_is_plausible(kind, lo, hi):
    torch = _torch()
    import paper_1908_06097_amd as shtx
    src = dst = None
    if kind.startswith("hbm"):
        src = torch.ones(1 << 26, dtype=torch.float32, device="cuda")  # 256 MiB
        dst = torch.empty_like(src) if kind == "hbm_copy" else None
    r = shtx.probe_peak(kind, src, dst)
    print(f"{kind}: {r:.1f}", flush=True)
    assert lo < r < hi, (kind, r)


def test_probe_rejects_host_and_overlapping_buffers():
    torch = _torch()
    import paper_1908_06097_amd as shtx
    lib = shtx.load_library()
    rate = ctypes.c_double(0.0)
    host = torch.ones(1 << 18, dtype=torch.float32)  # 1 MiB on the host
    dev = torch.ones(1 << 18, dtype=torch.float32, device="cuda")
    big = torch.empty(1 << 19, dtype=torch.float32, device="cuda")
    nb = ctypes.c_size_t(1 << 20)
    # host source or destination
    assert lib.shtx_probe_peak(6, ctypes.c_void_p(host.data_ptr()), ctypes.c_void_p(dev.data_ptr()), nb,
                               ctypes.byref(rate), None) == -1
    assert lib.shtx_probe_peak(5, ctypes.c_void_p(dev.data_ptr()), ctypes.c_void_p(host.data_ptr()), nb,
                               ctypes.byref(rate), None) == -1
    # overlapping copy, and a size below 1 MiB or not a multiple of 16
    assert lib.shtx_probe_peak(5, ctypes.c_void_p(big.data_ptr()), ctypes.c_void_p(big.data_ptr() + 1024), nb,
                               ctypes.byref(rate), None) == -1
    assert lib.shtx_probe_peak(6, ctypes.c_void_p(dev.data_ptr()), ctypes.c_void_p(big.data_ptr()),
                               ctypes.c_size_t(4096), ctypes.byref(rate), None) == -1
    assert lib.shtx_probe_peak(6, ctypes.c_void_p(dev.data_ptr()), ctypes.c_void_p(big.data_ptr()),
                               ctypes.c_size_t((1 << 20) + 8), ctypes.byref(rate), None) == -1
    torch.cuda.synchronize()
