"""Runtime behaviour of the HIP transforms: hipGraph replay, determinism,
exact scaling, field independence, NaN propagation, degenerate sizes and
argument errors.  Every call goes through the C ABI."""
import ctypes

import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu


def _env():
    import torch
    import paper_1908_06097_amd as shtx
    if not torch.cuda.is_available():
        pytest.fail("GPU test without a GPU")
    return torch, shtx


def _spec(torch, plan, key=21, fields=None):
    fields = range(plan.nfld) if fields is None else fields
    return torch.from_numpy(si.spectral_fields(plan.trunc, key, fields)).to(plan.complex_dtype).cuda()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3", "fp64"])
def test_graph_replay_matches_eager(prec):
    torch, shtx = _env()
    eager = shtx.Plan(63, "octahedral", 128, 5, prec)
    graphed = shtx.Plan(63, "octahedral", 128, 5, prec, graph=True)
    a = _spec(torch, eager)
    ref_g = eager.inv(a)
    ref_s = eager.dir(ref_g)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        a2 = a.clone()
        g = torch.empty_like(ref_g)
        s = torch.empty_like(ref_s)
        for rep in range(4):
            graphed.inv(a2, out=g)
            graphed.dir(g, out=s)
            side.synchronize()
            assert torch.equal(g, ref_g), rep
            assert torch.equal(s, ref_s), rep
            g.mul_(0.5)  # eager work on the same stream between replays
            s.zero_()
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["fp32", "fp16x3"])
def test_caller_graph_capture(prec):
    """A caller's own graph (torch.cuda.graph) captures a plan's transforms:
    every replay, with eager work on the same buffers between replays,
    equals the eager result bit for bit (the split-half form's per-field
    maxima are cleared by a kernel, so each replay starts from zero)."""
    torch, shtx = _env()
    plan = shtx.Plan(63, "octahedral", 128, 5, prec)
    a = _spec(torch, plan)
    ref_g = plan.inv(a)
    ref_s = plan.dir(ref_g)
    g = torch.empty_like(ref_g)
    s = torch.empty_like(ref_s)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up outside the capture
        plan.inv(a, out=g)
        plan.dir(g, out=s)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.inv(a, out=g)
        plan.dir(g, out=s)
    for rep in range(4):
        g.fill_(float("nan"))
        s.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(g, ref_g), rep
        assert torch.equal(s, ref_s), rep
    del graph
    torch.cuda.synchronize()


def test_two_plans_on_two_streams():
    """Two plans used at the same time from two streams give the results each
    gives alone (no state is shared between plans)."""
    torch, shtx = _env()
    pa = shtx.Plan(127, "octahedral", 256, 7, "fp32")
    pb = shtx.Plan(127, "octahedral", 256, 11, "fp16x3")
    a, b = _spec(torch, pa, key=41), _spec(torch, pb, key=42)
    ref_a = pa.dir(pa.inv(a))
    ref_b = pb.dir(pb.inv(b))
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    outs = []
    for _ in range(3):
        with torch.cuda.stream(s1):
            ra = pa.dir(pa.inv(a))
        with torch.cuda.stream(s2):
            rb = pb.dir(pb.inv(b))
        outs.append((ra, rb))
    torch.cuda.synchronize()
    for ra, rb in outs:
        assert torch.equal(ra, ref_a) and torch.equal(rb, ref_b)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x3"])
def test_graph_path_matches_oracle(prec):
    """The hipGraph replay path (the one the benchmark times) against the
    oracle on a multi-tile shape, every transform kind, four replays each."""
    from test_gpu_transforms import _check_all
    torch, shtx = _env()
    N, nlat, F = 159, 320, 70
    plan = shtx.Plan(N, "octahedral", nlat, F, prec, graph=True)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        print(f"graph path T{N} O{nlat // 2} F={F} {prec}", flush=True)
        _check_all(plan, N, plan.ring_lengths(), 11, range(F), prec)
        # replays of the cached graphs, with eager work between them, stay equal
        a = _spec(torch, plan, key=11)
        g0 = plan.inv(a).clone()
        s0 = plan.dir(g0).clone()
        g, s = torch.empty_like(g0), torch.empty_like(s0)
        for rep in range(4):
            plan.inv(a, out=g)
            plan.dir(g, out=s)
            side.synchronize()
            assert torch.equal(g, g0) and torch.equal(s, s0), rep
            g.add_(1.0)
            s.zero_()
    torch.cuda.synchronize()
    plan.close()


def test_bitwise_deterministic():
    torch, shtx = _env()
    plan = shtx.Plan(159, "octahedral", 320, 33, "fp32")
    a = _spec(torch, plan)
    g1, g2 = plan.inv(a), plan.inv(a)
    assert torch.equal(g1, g2)
    assert torch.equal(plan.dir(g1), plan.dir(g2))
    assert torch.equal(plan.inv_adj(g1), plan.inv_adj(g2))
    assert torch.equal(plan.dir_adj(a), plan.dir_adj(a))


def test_power_of_two_scaling_is_exact_and_zero_maps_to_zero():
    torch, shtx = _env()
    plan = shtx.Plan(95, "octahedral", 192, 4, "fp32")
    a = _spec(torch, plan)
    assert torch.equal(plan.inv(2 * a), 2 * plan.inv(a))
    g = plan.inv(a)
    assert torch.equal(plan.dir(0.25 * g), 0.25 * plan.dir(g))
    assert torch.count_nonzero(plan.inv(torch.zeros_like(a))) == 0
    assert torch.count_nonzero(plan.dir(torch.zeros_like(g))) == 0


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
def test_fields_are_independent(prec):
    torch, shtx = _env()
    plan = shtx.Plan(127, "octahedral", 256, 70, prec)
    a = _spec(torch, plan)
    b = a.clone()
    b[1:] = 0
    assert torch.equal(plan.inv(a)[0], plan.inv(b)[0])
    g = plan.inv(a)
    h = g.clone()
    h[1:] = 0
    assert torch.equal(plan.dir(g)[0], plan.dir(h)[0])


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
def test_nan_propagates_only_within_its_field(prec):
    """A NaN stays in its field in both directions (the split-half form's
    per-field scales are taken from a maximum that ignores or isolates it)."""
    torch, shtx = _env()
    plan = shtx.Plan(63, "octahedral", 128, 3, prec)
    a = _spec(torch, plan)
    a[1, 10] = float("nan")
    g = plan.inv(a)
    assert torch.isnan(g[1]).any()
    assert not torch.isnan(g[0]).any() and not torch.isnan(g[2]).any()
    g = plan.inv(_spec(torch, plan))
    g[2, 100] = float("nan")
    b = plan.dir(g)
    assert torch.isnan(torch.view_as_real(b[2])).any()
    assert not torch.isnan(torch.view_as_real(b[:2])).any()


# reduced-precision forms on the degenerate shapes: max relative error bounds
# (split IEEE half reaches FP32's accuracy)
DEGENERATE_TOL = {"fp32": 1e-5, "bf16x3": 1e-4, "fp16x3": 1e-5}


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("trunc,grid,nlat,nlon", [(0, "octahedral", 2, 0), (1, "octahedral", 4, 0),
                                                   (2, "full", 4, 6), (7, "full", 8, 16)])
def test_degenerate_sizes_reduced_precision(trunc, grid, nlat, nlon, prec):
    import oracle
    torch, shtx = _env()
    plan = shtx.Plan(trunc, grid, nlat, 3, prec, nlon_full=nlon)
    nl = plan.ring_lengths()
    a = si.spectral_fields(trunc, 32, [0, 1, 2])
    g = plan.inv(torch.from_numpy(a).to(torch.complex64).cuda()).double().cpu().numpy()
    ref = oracle.inv(trunc, nl, a)
    tol = DEGENERATE_TOL[prec]
    assert np.max(np.abs(g - ref)) <= tol * np.max(np.abs(ref)), np.max(np.abs(g - ref)) / np.max(np.abs(ref))
    b = plan.dir(torch.from_numpy(ref).float().cuda()).cpu().numpy().astype(np.complex128)
    bref = oracle.dir(trunc, nl, ref)
    assert np.max(np.abs(b - bref)) <= tol * np.max(np.abs(bref)), np.max(np.abs(b - bref)) / np.max(np.abs(bref))


@pytest.mark.parametrize("trunc,grid,nlat,nlon", [(0, "octahedral", 2, 0), (1, "octahedral", 4, 0),
                                                   (2, "full", 4, 6), (7, "full", 8, 16)])
def test_degenerate_sizes_fp64(trunc, grid, nlat, nlon):
    import oracle
    torch, shtx = _env()
    plan = shtx.Plan(trunc, grid, nlat, 2, "fp64", nlon_full=nlon)
    nl = plan.ring_lengths()
    a = si.spectral_fields(trunc, 31, [0, 1])
    g = plan.inv(torch.from_numpy(a).cuda()).cpu().numpy()
    ref = oracle.inv(trunc, nl, a)
    assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref))
    b = plan.dir(torch.from_numpy(ref).cuda()).cpu().numpy()
    bref = oracle.dir(trunc, nl, ref)
    assert np.max(np.abs(b - bref)) <= 1e-12 * np.max(np.abs(bref))


def test_plan_info_and_geometry():
    torch, shtx = _env()
    plan = shtx.Plan(255, "octahedral", 512, 7, "fp32")
    info = plan.info
    assert info.nspec == 256 * 257 // 2
    assert info.npts == int(plan.ring_lengths().sum()) == 271360
    assert info.nfour == 100568
    assert info.max_nlon == 1040 and info.table_bytes > 0 and info.legendre_flops > 0


def test_argument_errors():
    torch, shtx = _env()
    plan = shtx.Plan(31, "octahedral", 64, 2, "fp32")
    a = _spec(torch, plan)
    with pytest.raises(shtx.ShtxError):
        plan.inv(a.to(torch.complex128))
    with pytest.raises(shtx.ShtxError):
        plan.inv(a[:1])
    with pytest.raises(shtx.ShtxError):
        plan.inv(a.cpu())
    with pytest.raises(shtx.ShtxError):  # host output tensor: refused before any launch
        plan.inv(a, out=torch.empty((plan.nfld, plan.npts), dtype=torch.float32))
    lib = shtx.load_library()
    # a host pointer through the C ABI is refused by the library itself
    host = np.zeros(plan.npts * plan.nfld + 16, dtype=np.float32)
    hp = ctypes.c_void_p((host.ctypes.data + 15) // 16 * 16)
    assert lib.shtx_inv_trans(plan._h, ctypes.c_void_p(a.data_ptr()), hp, None) == -1
    assert lib.shtx_dir_trans(plan._h, hp, ctypes.c_void_p(a.data_ptr()), None) == -1
    buf = torch.zeros(max(plan.npts, 2 * plan.nspec) * 2, dtype=torch.float32, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    rc = lib.shtx_inv_trans(plan._h, p, p, None)  # output overlaps input
    assert rc == -1
    assert lib.shtx_plan_legendre(plan._h, 32, None) == -1


def _library_loaded(shtx):
    """Create and destroy one small plan, so that the library's code objects
    (and its static scratch array) are resident before a memory baseline."""
    shtx.Plan(15, "octahedral", 32, 1, "fp32").close()


def test_plan_create_destroy_cycles():
    torch, shtx = _env()
    _library_loaded(shtx)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(5):
        p = shtx.Plan(255, "octahedral", 512, 16, "bf16x3")
        p.close()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 >= free0 - (64 << 20)


def test_plan_beyond_device_memory_fails_cleanly():
    """A plan whose Fourier workspace cannot fit in HBM (TCo1279, 8000 fields
    in FP64: about 316 GB) fails with SHTX_ENOMEM, frees what it had
    allocated (tables included) and leaves the device usable."""
    torch, shtx = _env()
    _library_loaded(shtx)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    with pytest.raises(shtx.ShtxError) as err:
        shtx.Plan(1279, "octahedral", 2560, 8000, "fp64")
    assert "out of memory" in str(err.value), str(err.value)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 >= free0 - (64 << 20), (free0, free1)
    plan = shtx.Plan(31, "octahedral", 64, 2, "fp64")
    a = _spec(torch, plan)
    assert torch.isfinite(torch.view_as_real(plan.dir(plan.inv(a)))).all()
    plan.close()
