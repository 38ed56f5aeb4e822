"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# Largest LDS complex values per FFT block (single-precision FFTs also serve
# BF16x3) and the autotuner's other two blockings.
FFT_CAPS = {"fp32": (8192, 4096, 2730), "bf16x3": (8192, 4096, 2730), "fp16x3": (8192, 4096, 2730),
            "fp64": (8192, 4096, 2730)}


def _declared():
    src = open(os.path.join(ROOT, "include", "shtx.h")).read()
    return sorted(set(re.findall(r"\b(shtx_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_1908_06097_amd as shtx
    if not os.path.exists(shtx.LIB_PATH):
        pytest.fail("libshtx.so is not built (run __graft_entry__.build())")
    return shtx.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "shtx_inv_trans" in names and "shtx_dir_trans_adj" in names
    for n in names:
        assert hasattr(lib, n), n


def test_probe_peak_rejects_bad_arguments_before_any_launch(lib):
    import ctypes
    rate = ctypes.c_double(1.0)
    # unknown kinds and a missing result pointer are refused on the host
    assert lib.shtx_probe_peak(-1, None, None, 0, ctypes.byref(rate), None) == -1
    assert lib.shtx_probe_peak(7, None, None, 0, ctypes.byref(rate), None) == -1
    assert lib.shtx_probe_peak(1, None, None, 0, None, None) == -1


def test_strerror(lib):
    assert lib.shtx_strerror(0) == b"success"
    assert lib.shtx_strerror(-1) == b"invalid argument"
    assert lib.shtx_strerror(-4) == b"unsupported configuration"


@pytest.mark.parametrize("args,code", [
    ((-1, 1, 64, 0, 1, 1), -1),        # negative truncation
    ((31, 1, 64, 0, 0, 1), -1),        # no fields
    ((31, 7, 64, 0, 1, 1), -1),        # unknown grid
    ((31, 1, 64, 0, 1, 9), -1),        # unknown precision
    ((31, 1, 63, 0, 1, 1), -4),        # odd number of latitudes
    ((31, 0, 64, 127, 1, 1), -4),      # odd ring length on a full grid
    ((31, 0, 64, 0, 1, 1), -1),        # full grid without a ring length
])
def test_plan_create_rejects_bad_arguments(lib, args, code):
    h = ctypes.c_void_p()
    rc = lib.shtx_plan_create(ctypes.byref(h), *args, 0, None)
    assert rc == code
    assert not h.value


def test_null_handles(lib):
    assert lib.shtx_plan_create(None, 31, 1, 64, 0, 1, 1, 0, None) == -1
    assert lib.shtx_inv_trans(None, None, None, None) == -1
    assert lib.shtx_plan_destroy(None) == -1
    assert lib.shtx_plan_info(None, None) == -1


def test_python_binding_refuses_without_gpu():
    torch = pytest.importorskip("torch")
    import paper_1908_06097_amd as shtx
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(shtx.ShtxError):
        shtx.Plan(31, "octahedral", 64, 1, "fp32")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x3"])
def test_plan_check_all_workloads(lib, prec):
    """Host dry run of every workload's plan: geometry and every kernel's
    launch shape pass the library's own bounds checks, without a GPU."""
    import paper_1908_06097_amd as shtx
    import synth_inputs as si
    sizes = {"t79_full": (3240, 51200, 12800), "t255_o256": (32896, 271360, 100568),
             "t399_o400": (80200, 654400, 243560), "tco639_o640": (205120, 1661440, 620120),
             "tco1279_o1280": (819840, 6599680, 2469080), "tco1999_o2000": (2001000, 16072000, None)}
    for key, w in si.WORKLOADS.items():
        if key in ("tco1279_o1280", "tco1999_o2000") and prec != "fp32":
            continue  # same layout code; keep the CPU suite short
        rc, info = shtx.plan_check(w.trunc, w.grid, w.nlat, w.nfld, prec, w.nlon_full)
        assert rc == 0, (key, prec, rc)
        ns, npts, nfour = sizes[key]
        assert (info.nspec, info.npts) == (ns, npts)
        nlon = w.ring_lengths()
        assert info.nfour == int(sum(min(w.trunc, (int(n) - 1) // 2) + 1 for n in nlon))
        if nfour is not None:
            assert info.nfour == nfour
        assert info.table_bytes > 0 and info.legendre_flops > 0


def test_plan_check_rejects(lib):
    import paper_1908_06097_amd as shtx
    assert shtx.plan_check(31, "octahedral", 63)[0] == -4
    assert shtx.plan_check(-1, "octahedral", 64)[0] == -1
    assert shtx.plan_check(31, "full", 64, nlon_full=0)[0] == -1


@pytest.mark.parametrize("prec,shapes", [("fp32", [(128, 128), (64, 128), (128, 64)]),
                                         ("fp64", [(64, 64), (32, 64), (64, 32)]),
                                         ("bf16x3", [(128, 128), (64, 128)]),
                                         ("fp16x3", [(128, 128), (64, 128)])])
def test_plan_check_every_tuning_shape(lib, prec, shapes):
    """Every tile shape and FFT blocking the autotuner may pick passes the
    library's launch-shape checks on the workloads (host dry run)."""
    import paper_1908_06097_amd as shtx
    import synth_inputs as si
    for key in ("t255_o256", "t399_o400"):
        w = si.WORKLOADS[key]
        for t in shapes:
            # the autotuner's FFT blockings: the precision's LDS cap, 1/2 and 1/3 of it
            for cap in FFT_CAPS[prec]:
                rc, info = shtx.plan_check_shapes(w.trunc, w.grid, w.nlat, w.nfld, prec, t, t, cap, w.nlon_full)
                assert rc == 0, (key, prec, t, cap, rc)
                assert tuple(info.inv_tile) == t and tuple(info.dir_tile) == t and info.fft_cap == cap


def test_plan_check_shapes_rejects(lib):
    import paper_1908_06097_amd as shtx
    assert shtx.plan_check_shapes(255, "octahedral", 512, 7, "fp32", (96, 128), (128, 128), 6144)[0] == -4
    assert shtx.plan_check_shapes(255, "octahedral", 512, 7, "fp32", (64, 64), (128, 128), 6144)[0] == -4
    assert shtx.plan_check_shapes(255, "octahedral", 512, 7, "fp64", (128, 128), (64, 64), 6144)[0] == -4
    assert shtx.plan_check_shapes(255, "octahedral", 512, 7, "fp32", (128, 128), (128, 128), 0)[0] == -1
    assert shtx.plan_check_shapes(255, "octahedral", 512, 7, "fp32", (128, 128), (128, 128), FFT_CAPS["fp32"][0] + 1)[0] == -1
    assert shtx.plan_check_shapes(255, "octahedral", 512, 7, "fp64", (64, 64), (64, 64), FFT_CAPS["fp64"][0] + 1)[0] == -1
