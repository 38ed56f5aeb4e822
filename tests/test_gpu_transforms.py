"""GPU parity of the HIP transforms against the FP64 CPU oracle.

Every call goes through the C ABI (via the thin Python binding).  Inputs are
the seeded synthetic spectra of ``synth_inputs``; expected values come only
from ``oracle``.  Tolerances: FP64 1e-12 (max relative), FP32 1e-5 (RMS),
split BF16 1e-4 (RMS), split IEEE half 2e-6 (RMS), per field, on spectral
and grid outputs.
"""
import numpy as np
import pytest

import synth_inputs as si
from error_metrics import grid_errors, spec_errors

pytestmark = pytest.mark.gpu

# split IEEE half keeps 22 of FP32's 24 significand bits on every operand,
# so its bound is set well inside FP32's: an inexact split (a hi and lo that
# do not sum to the operand) shows up at 1e-5 and above
TOL_RMS = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4, "fp16x3": 2e-6}
TOL_MAX = {"fp64": 1e-12, "fp32": 1e-4, "bf16x3": 1e-3, "fp16x3": 1e-5}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test without a GPU")
    return torch


def _shtx():
    import paper_1908_06097_amd as shtx
    return shtx


def _oracle():
    import oracle
    return oracle


def _dev(x, dtype):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def _np(t):
    return t.detach().cpu().numpy()


def _say(*a):
    print(*a, flush=True)


# ---------------------------------------------------------------------------
# Plan-time data: nodes and tables
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nlat", [160, 512, 1280, 2560])
def test_nodes_bitwise(nlat):
    shtx, o = _shtx(), _oracle()
    _say(f"nodes nlat={nlat}")
    plan = shtx.Plan(15, "octahedral", nlat, 1, "fp64")
    mu, w = plan.nodes()
    mu_o, w_o = o.gauss(nlat)
    assert np.array_equal(mu, mu_o), np.flatnonzero(mu != mu_o)[:10]
    assert np.all(np.abs(w - w_o) <= np.spacing(w_o)), np.max(np.abs(w - w_o) / np.spacing(w_o))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-7), ("bf16x3", 1.5e-5), ("fp16x3", 1e-6)])
def test_legendre_tables(prec, tol):
    shtx, o = _shtx(), _oracle()
    N, nlat = 255, 512
    _say(f"tables T{N} O{nlat // 2} {prec}")
    plan = shtx.Plan(N, "octahedral", nlat, 1, prec)
    mu, _ = plan.nodes()
    nlon = plan.ring_lengths()
    for m in (0, 1, 17, 128, 200, 255):
        tab = plan.legendre(m)
        rings = [j for j in range(nlat // 2) if o.ring_cutoff(N, nlon[j]) >= m]
        assert tab.shape == (len(rings), N - m + 1)
        ref = o.legendre(N, m, mu[rings])
        err = np.abs(tab - ref).max() / np.abs(ref).max()
        assert err < tol, (m, err)


def test_legendre_tables_beyond_double_range():
    """TCo1999 (N = 1999 on O2000) FP64 tables: wavenumbers whose sectoral
    seeds fall below 1e-310 on many rings while P̄_n^m there reaches order one
    (up to about 5) match the oracle's extended-exponent columns."""
    shtx, o = _shtx(), _oracle()
    N, nlat = 1999, 4000
    _say(f"tables T{N} O{nlat // 2} fp64 (extended exponent)")
    plan = shtx.Plan(N, "octahedral", nlat, 1, "fp64")
    mu, _ = plan.nodes()
    nlon = plan.ring_lengths()
    for m in (700, 862, 940):
        tab = plan.legendre(m)
        rings = [j for j in range(nlat // 2) if o.ring_cutoff(N, nlon[j]) >= m]
        ref = o.legendre(N, m, mu[rings])
        s = np.sqrt((1 - mu[rings]) * (1 + mu[rings]))
        k = np.arange(1, m + 1)
        log_seed = np.sum(0.5 * np.log10((2 * k + 1) / (2 * k))) + m * np.log10(s)
        low = log_seed < -310
        assert low.any() and np.abs(ref[low]).max() > 1.0, m  # the case is exercised
        err = np.abs(tab - ref).max() / np.abs(ref).max()
        _say(f"  m={m}: {int(low.sum())} rings with seeds < 1e-310, max |P| there "
             f"{np.abs(ref[low]).max():.2f}, error {err:.2e}")
        assert err < 1e-12, (m, err)
    plan.close()


# ---------------------------------------------------------------------------
# Transforms on small and multi-tile shapes
# ---------------------------------------------------------------------------

def _check_all(plan, N, nlon, key, fields, prec):
    torch, o = _torch(), _oracle()
    mu, w = o.gauss(len(nlon))
    a = si.spectral_fields(N, key, fields)
    nf = len(fields)
    g_ref = o.inv(N, nlon, a)
    spec = _dev(a, plan.complex_dtype)
    g = plan.inv(spec)
    em, er = grid_errors(_np(g), g_ref, nlon, w)
    _say(f"  inv   e_max {em.max():.2e} e_rms {er.max():.2e}")
    assert er.max() < TOL_RMS[prec] and em.max() < TOL_MAX[prec]

    b_ref = o.dir(N, nlon, g_ref)
    b = plan.dir(_dev(g_ref, plan.real_dtype))
    em, er = spec_errors(_np(b), b_ref, N)
    _say(f"  dir   e_max {em.max():.2e} e_rms {er.max():.2e}")
    assert er.max() < TOL_RMS[prec] and em.max() < TOL_MAX[prec]

    y = np.stack([si.white_noise_grid(int(nlon.sum()), 500 + f) for f in range(nf)])
    c_ref = o.inv_adj(N, nlon, y)
    c = plan.inv_adj(_dev(y, plan.real_dtype))
    em, er = spec_errors(_np(c), c_ref, N)
    _say(f"  iadj  e_max {em.max():.2e} e_rms {er.max():.2e}")
    assert er.max() < TOL_RMS[prec] and em.max() < TOL_MAX[prec]

    d_ref = o.dir_adj(N, nlon, a)
    d = plan.dir_adj(spec)
    em, er = grid_errors(_np(d), d_ref, nlon, w)
    _say(f"  dadj  e_max {em.max():.2e} e_rms {er.max():.2e}")
    assert er.max() < TOL_RMS[prec] and em.max() < TOL_MAX[prec]
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("shape", ["T31_O32_F3", "T63_full_F2", "T159_O160_F70"])
def test_transform_parity(prec, shape):
    shtx, o = _shtx(), _oracle()
    if shape == "T31_O32_F3":
        N, grid, nlat, nl_full, F = 31, "octahedral", 64, 0, 3
    elif shape == "T63_full_F2":
        N, grid, nlat, nl_full, F = 63, "full", 64, 128, 2
    else:
        N, grid, nlat, nl_full, F = 159, "octahedral", 320, 0, 70
    _say(f"parity {shape} {prec}")
    plan = shtx.Plan(N, grid, nlat, F, prec, nlon_full=nl_full)
    nlon = plan.ring_lengths()
    _check_all(plan, N, nlon, 11, range(F), prec)


# Full grids of one ring length each, one per kind of ring FFT plan: half
# lengths h = 2 p with a prime p above 191 (a matrix-core prime pass up to the
# cost model's crossover), a prime above the crossover (Bluestein), two large
# primes, a small prime with a large smooth cofactor, and odd half lengths
# (h = 211, a single prime butterfly; h = 1021, Bluestein), where the chirp at
# h - m is minus the chirp at m.
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nlon", [844, 1604, 2452, 3596, 4084, 5180, 422, 2042])
def test_ring_kinds_parity(prec, nlon):
    shtx = _shtx()
    N, nlat, F = 31, 16, 3
    _say(f"ring kinds nlon={nlon} {prec}")
    plan = shtx.Plan(N, "full", nlat, F, prec, nlon_full=nlon)
    _check_all(plan, N, plan.ring_lengths(), 13, range(F), prec)


# Legendre GEMM column tiling: 128 columns exactly (64 fields), a last tile at
# most half used (70 fields: covered by the 64-column tail launch) and one
# more than half used (100 fields: no tail).
@pytest.mark.parametrize("F", [64, 70, 100])
def test_gemm_column_tiles_fp32(F):
    shtx = _shtx()
    N, nlat = 63, 128
    _say(f"column tiles F={F}")
    plan = shtx.Plan(N, "octahedral", nlat, F, "fp32")
    _check_all(plan, N, plan.ring_lengths(), 17, range(F), "fp32")


def test_t79_full_fp64_round_trip():
    """T79 on the full 160 x 320 grid, 1 field, FP64: parity and round trip <= 1e-12."""
    shtx, o = _shtx(), _oracle()
    wl = si.WORKLOADS["t79_full"]
    plan = shtx.Plan(wl.trunc, "full", wl.nlat, 1, "fp64", nlon_full=wl.nlon_full)
    nlon = plan.ring_lengths()
    a = si.spectral_fields(wl.trunc, wl.key, [0])
    _check_all(plan, wl.trunc, nlon, wl.key, [0], "fp64")
    b = _np(plan.dir(plan.inv(_dev(a, plan.complex_dtype))))
    em, er = spec_errors(b, a, wl.trunc)
    _say(f"  round trip e_max {em.max():.2e} e_rms {er.max():.2e}")
    assert em.max() < 1e-12 and er.max() < 1e-12


# ---------------------------------------------------------------------------
# Wind images from vorticity and divergence
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("shape", ["T31_O32_F3", "T159_O160_F35", "T63_full_F2"])
def test_uv_parity(prec, shape):
    """U = u cos(phi) and V = v cos(phi) from random band-limited vorticity and
    divergence against the oracle (a plan of truncation N + 1, 2 F fields)."""
    torch, shtx, o = _torch(), _shtx(), _oracle()
    if shape == "T31_O32_F3":
        N, grid, nlat, nl_full, F = 31, "octahedral", 64, 0, 3
    elif shape == "T159_O160_F35":
        N, grid, nlat, nl_full, F = 159, "octahedral", 320, 0, 35
    else:
        N, grid, nlat, nl_full, F = 63, "full", 64, 130, 2
    _say(f"uv {shape} {prec}")
    plan = shtx.Plan(N + 1, grid, nlat, 2 * F, prec, nlon_full=nl_full, uv=True)
    nlon = plan.ring_lengths()
    _, w = o.gauss(nlat)
    zeta = si.spectral_fields(N, 61, range(F))
    dvg = si.spectral_fields(N, 62, range(F))
    ref = o.uv(N, nlon, zeta, dvg)
    g = _np(plan.uv(_dev(zeta, plan.complex_dtype), _dev(dvg, plan.complex_dtype)))
    em, er = grid_errors(g, ref, nlon, w)
    _say(f"  U,V e_max {em.max():.2e} e_rms {er.max():.2e}")
    assert er.max() < TOL_RMS[prec] and em.max() < TOL_MAX[prec]
    plan.close()


def test_uv_graph_replay_and_gradient():
    """The wind transform replays as a graph; with zeta = 0 and D = -n(n+1) s it
    gives the gradient (d s/d lambda, (1 - mu^2) d s/d mu) of a scalar s, which
    for s = P̄_2^0 = (sqrt(5)/2)(3 mu^2 - 1) is (0, 3 sqrt(5) mu (1 - mu^2))."""
    torch, shtx, o = _torch(), _shtx(), _oracle()
    N, F = 31, 2
    plan = shtx.Plan(N + 1, "octahedral", 64, 2 * F, "fp64", uv=True, graph=True)
    ns = si.nspec(N)
    s_spec = np.zeros((F, ns), complex)
    s_spec[:, 2] = 1.0  # (m, n) = (0, 2)
    m_, n_ = si.spec_mn(N)
    dvg = -(n_ * (n_ + 1))[None, :] * s_spec
    zeta = np.zeros_like(dvg)
    mu, _ = plan.nodes()
    nlon = plan.ring_lengths()
    x = np.repeat(mu, nlon)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        vz, vd = _dev(zeta, torch.complex128), _dev(dvg, torch.complex128)
        out = torch.empty((2 * F, plan.npts), dtype=torch.float64, device="cuda")
        for rep in range(3):
            out.fill_(float("nan"))
            plan.uv(vz, vd, out=out)
            side.synchronize()
            g = _np(out)
            assert np.max(np.abs(g[:F])) < 1e-13, rep
            V = 3 * np.sqrt(5) * x * (1 - x * x)
            assert np.max(np.abs(g[F:] - V[None, :])) < 1e-13, rep
    torch.cuda.synchronize()
    plan.close()


# ---------------------------------------------------------------------------
# Full-size workloads on sampled fields
# ---------------------------------------------------------------------------

# Fixed, spread samples of the 411 fields the oracle checks one by one.
SAMPLE_16 = list(range(0, 411, 26))   # TCo1279: 0, 26, ..., 390
SAMPLE_32 = list(range(0, 411, 13))   # TCo639: 0, 13, ..., 403
_ORACLE_CACHE = {}


def _oracle_of(wl, what, fields):
    """Oracle outputs on the sampled fields, computed once per session and
    shared by every precision's test of the workload."""
    key = (wl.name, what, tuple(fields))
    if key not in _ORACLE_CACHE:
        o = _oracle()
        nlon = wl.ring_lengths()
        a = si.spectral_fields(wl.trunc, wl.key, fields)
        if what == "inv":
            r = o.inv(wl.trunc, nlon, a)
        elif what == "dir":
            r = o.dir(wl.trunc, nlon, _oracle_of(wl, "inv", fields))
        elif what == "noise":
            r = np.stack([si.white_noise_grid(int(nlon.sum()), 500 + f) for f in fields])
        elif what == "inv_adj":
            r = o.inv_adj(wl.trunc, nlon, _oracle_of(wl, "noise", fields))
        elif what == "dir_adj":
            r = o.dir_adj(wl.trunc, nlon, a)
        else:
            raise ValueError(what)
        _ORACLE_CACHE[key] = r
    return _ORACLE_CACHE[key]


def _rows_on_device(torch, plan, rows, sample, nfld):
    """[nfld, n] device array: the sampled fields hold `rows`, every other field
    a copy of the first row (built on the device, not in host memory)."""
    dt = plan.real_dtype if not np.iscomplexobj(rows) else plan.complex_dtype
    first = torch.from_numpy(np.ascontiguousarray(rows[:1])).to(dt).cuda()
    out = first.expand(nfld, -1).contiguous()
    out[list(sample)] = torch.from_numpy(np.ascontiguousarray(rows)).to(dt).cuda()
    return out


def _full_size(key, prec, sample, adjoints=False, forward=True):
    """inv and dir (and, with adjoints=True, inv_adj and dir_adj) of the whole
    workload on the device, compared field by field with the oracle on the
    sampled fields: max and RMS errors (the metrics of error_metrics)."""
    torch, shtx, o = _torch(), _shtx(), _oracle()
    wl = si.WORKLOADS[key]
    sample = list(sample)
    _say(f"{wl.name} {prec}: F={wl.nfld}, {len(sample)} sampled fields {sample[:4]}...")
    plan = shtx.Plan(wl.trunc, wl.grid, wl.nlat, wl.nfld, prec, nlon_full=wl.nlon_full)
    nlon = plan.ring_lengths()
    _, w = o.gauss(wl.nlat)
    a_all = si.spectral_fields(wl.trunc, wl.key, range(wl.nfld))
    spec = _dev(a_all, plan.complex_dtype)
    del a_all
    a = si.spectral_fields(wl.trunc, wl.key, sample)
    tol_r, tol_m = TOL_RMS[prec], TOL_MAX[prec]
    if forward:
        g = _np(plan.inv(spec)[sample])
        em, er = grid_errors(g, _oracle_of(wl, "inv", sample), nlon, w)
        _say(f"  inv   e_max {em.max():.2e} e_rms {er.max():.2e} (median e_rms {np.median(er):.2e})")
        assert er.max() < tol_r and em.max() < tol_m
        # direct transform of band-limited oracle grids in the sampled slots
        g_in = _rows_on_device(torch, plan, _oracle_of(wl, "inv", sample), sample, wl.nfld)
        b = _np(plan.dir(g_in)[sample])
        del g_in
        em, er = spec_errors(b, _oracle_of(wl, "dir", sample), wl.trunc)
        _say(f"  dir   e_max {em.max():.2e} e_rms {er.max():.2e} (median e_rms {np.median(er):.2e})")
        assert er.max() < tol_r and em.max() < tol_m
        # round trip on the device, compared with the seeded input
        b = _np(plan.dir(plan.inv(spec))[sample])
        em, er = spec_errors(b, a, wl.trunc)
        _say(f"  round trip vs input e_max {em.max():.2e} e_rms {er.max():.2e}")
        assert er.max() < max(tol_r, 1e-12) * 4
    if adjoints:
        y = _rows_on_device(torch, plan, _oracle_of(wl, "noise", sample), sample, wl.nfld)
        c = _np(plan.inv_adj(y)[sample])
        del y
        em, er = spec_errors(c, _oracle_of(wl, "inv_adj", sample), wl.trunc)
        _say(f"  iadj  e_max {em.max():.2e} e_rms {er.max():.2e} (median e_rms {np.median(er):.2e})")
        assert er.max() < tol_r and em.max() < tol_m
        d = _np(plan.dir_adj(spec)[sample])
        em, er = grid_errors(d, _oracle_of(wl, "dir_adj", sample), nlon, w)
        _say(f"  dadj  e_max {em.max():.2e} e_rms {er.max():.2e} (median e_rms {np.median(er):.2e})")
        assert er.max() < tol_r and em.max() < tol_m
    plan.close()
    torch.cuda.synchronize()


def test_t255_o256_fp32_411_fields():
    _full_size("t255_o256", "fp32", [0, 1, 137, 274, 410], adjoints=True)


def test_t255_o256_fp64_411_fields():
    _full_size("t255_o256", "fp64", [0, 205, 410], adjoints=True)


def test_tco639_o640_bf16x3_411_fields():
    _full_size("tco639_o640", "bf16x3", SAMPLE_32)


def test_tco1279_o1280_fp32_411_fields():
    _full_size("tco1279_o1280", "fp32", SAMPLE_16)


def test_tco1279_o1280_fp32_adjoints():
    _full_size("tco1279_o1280", "fp32", SAMPLE_16, adjoints=True, forward=False)


def test_tco1279_o1280_bf16x3_411_fields():
    _full_size("tco1279_o1280", "bf16x3", SAMPLE_16)


def test_tco1279_o1280_bf16x3_adjoints():
    _full_size("tco1279_o1280", "bf16x3", SAMPLE_16, adjoints=True, forward=False)


def test_tco639_o640_fp16x3_411_fields():
    _full_size("tco639_o640", "fp16x3", SAMPLE_32)


def test_tco1279_o1280_fp16x3_411_fields():
    _full_size("tco1279_o1280", "fp16x3", SAMPLE_16, adjoints=True)


def _sampled_size(key, prec, sample):
    """Like _full_size for a workload too large to generate on the host: the
    device arrays hold the sampled fields' seeded rows and copies of the
    first one elsewhere (fields are independent); inverse, direct of the
    oracle's band-limited grids, and the device round trip, on the samples."""
    torch, shtx, o = _torch(), _shtx(), _oracle()
    wl = si.WORKLOADS[key]
    sample = list(sample)
    _say(f"{wl.name} {prec}: F={wl.nfld}, sampled fields {sample}")
    plan = shtx.Plan(wl.trunc, wl.grid, wl.nlat, wl.nfld, prec, nlon_full=wl.nlon_full)
    nlon = plan.ring_lengths()
    _, w = o.gauss(wl.nlat)
    a = si.spectral_fields(wl.trunc, wl.key, sample)
    spec = _rows_on_device(torch, plan, a, sample, wl.nfld)
    g_ref = o.inv(wl.trunc, nlon, a)
    g = _np(plan.inv(spec)[sample])
    em, er = grid_errors(g, g_ref, nlon, w)
    _say(f"  inv   e_max {em.max():.2e} e_rms {er.max():.2e}")
    assert er.max() < TOL_RMS[prec] and em.max() < TOL_MAX[prec]
    del g
    b_ref = o.dir(wl.trunc, nlon, g_ref)
    g_in = _rows_on_device(torch, plan, g_ref, sample, wl.nfld)
    b = _np(plan.dir(g_in)[sample])
    del g_in
    em, er = spec_errors(b, b_ref, wl.trunc)
    _say(f"  dir   e_max {em.max():.2e} e_rms {er.max():.2e}")
    assert er.max() < TOL_RMS[prec] and em.max() < TOL_MAX[prec]
    b = _np(plan.dir(plan.inv(spec))[sample])
    em, er = spec_errors(b, a, wl.trunc)
    _say(f"  round trip vs input e_max {em.max():.2e} e_rms {er.max():.2e}")
    assert er.max() < max(TOL_RMS[prec], 1e-12) * 4
    plan.close()
    torch.cuda.synchronize()


def test_tco1999_o2000_fp32_411_fields():
    """The 5 km case (rings up to 8016 points, seeds below the double range)."""
    _sampled_size("tco1999_o2000", "fp32", [0, 137, 274, 410])


def test_tco1279_o1280_fp64_411_fields():
    _full_size("tco1279_o1280", "fp64", SAMPLE_16)
