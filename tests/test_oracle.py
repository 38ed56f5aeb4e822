"""Pins for the FP64 CPU oracle against facts fixed by mathematics.

Nothing here compares the oracle with itself: every check is a closed form, an
exactness property of Gauss quadrature, an independent library routine
(numpy, scipy) or a brute-force evaluation.  Each is chosen so that a likely
slip in the oracle (a dropped c_m, a wrong sign on sin, a swapped recurrence
coefficient, a transposed index, a wrong weight) fails at least one of them.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _orc():
    import oracle
    return oracle


# --------------------------------------------------------------------------
# Gauss-Legendre nodes and weights
# --------------------------------------------------------------------------

def test_gauss_closed_forms():
    o = _orc()
    mu, w = o.gauss(1)
    assert mu[0] == 0.0 and abs(w[0] - 2.0) < 1e-15
    mu, w = o.gauss(2)
    assert np.allclose(mu, [1 / math.sqrt(3), -1 / math.sqrt(3)], rtol=0, atol=2e-16)
    assert np.allclose(w, [1.0, 1.0], rtol=0, atol=2e-16)
    mu, w = o.gauss(3)
    assert np.allclose(mu, [math.sqrt(0.6), 0.0, -math.sqrt(0.6)], rtol=0, atol=2e-16)
    assert np.allclose(w, [5 / 9, 8 / 9, 5 / 9], rtol=0, atol=3e-16)
    # nlat = 4: mu = +-sqrt(3/7 -+ 2/7 sqrt(6/5)), w = (18 +- sqrt 30) / 36
    mu, w = o.gauss(4)
    a = math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5))
    b = math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5))
    assert np.allclose(mu, [b, a, -a, -b], rtol=0, atol=3e-16)
    assert np.allclose(w, [(18 - math.sqrt(30)) / 36, (18 + math.sqrt(30)) / 36,
                           (18 + math.sqrt(30)) / 36, (18 - math.sqrt(30)) / 36], rtol=0, atol=3e-16)


@pytest.mark.parametrize("nlat", [8, 33, 160, 512, 1280])
def test_gauss_quadrature_exactness(nlat):
    """Sum w = 2, exact monomial integrals up to degree 2 nlat - 1, symmetry."""
    o = _orc()
    mu, w = o.gauss(nlat)
    assert abs(w.sum() - 2.0) < 1e-14
    assert np.all(np.diff(mu) < 0)
    assert np.array_equal(mu[::-1], -mu)
    assert np.array_equal(w[::-1], w)
    for k in range(1, min(nlat, 40)):
        exact = 2.0 / (2 * k + 1)
        assert abs(np.sum(w * mu ** (2 * k)) - exact) < 2e-14, k
        assert abs(np.sum(w * mu ** (2 * k - 1))) < 1e-14


@pytest.mark.parametrize("nlat", [5, 64, 160, 199])
def test_gauss_vs_numpy_leggauss(nlat):
    o = _orc()
    mu, w = o.gauss(nlat)
    x, wl = np.polynomial.legendre.leggauss(nlat)
    x, wl = x[::-1], wl[::-1]
    ulp = np.spacing(np.abs(mu) + 1e-300)
    assert np.all(np.abs(mu - x) <= 4 * np.maximum(ulp, 1e-17))
    # numpy's weights are themselves only good to ~1e-11 near the poles; the
    # 60-digit check below pins the oracle's weights to an ulp.
    assert np.max(np.abs(w - wl) / wl) < 1e-10


def _legendre_decimal(n, x):
    p0, p1 = Decimal(1), x
    for l in range(2, n + 1):
        p0, p1 = p1, ((2 * l - 1) * x * p1 - (l - 1) * p0) / l
    return p1


@pytest.mark.parametrize("nlat,nodes", [(7, None), (64, None), (160, None),
                                        (2560, [0, 1, 2, 3, 640, 1279])])
def test_gauss_nodes_correctly_rounded(nlat, nodes):
    """Each node is the double nearest to the true root: P_nlat changes sign
    between the two half-ulp midpoints around it (50-digit decimal arithmetic)."""
    o = _orc()
    getcontext().prec = 60
    mu, _ = o.gauss(nlat)
    idx = range((nlat + 1) // 2) if nodes is None else nodes
    for j in idx:
        x = float(mu[j])
        if x == 0.0:
            assert nlat % 2 == 1
            continue
        h = Decimal(np.spacing(x)) / 2
        lo = _legendre_decimal(nlat, Decimal(x) - h)
        hi = _legendre_decimal(nlat, Decimal(x) + h)
        assert (lo > 0) != (hi > 0), (nlat, j)


@pytest.mark.parametrize("nlat", [64, 513])
def test_gauss_weights_high_precision(nlat):
    """w_j = 2 / ((1 - x^2) P'(x)^2) at the root refined in 60-digit decimal."""
    o = _orc()
    getcontext().prec = 60
    mu, w = o.gauss(nlat)
    for j in (0, 1, nlat // 4, nlat // 2 - 1):
        X = Decimal(float(mu[j]))
        for _ in range(3):
            p = _legendre_decimal(nlat, X)
            p1 = _legendre_decimal(nlat - 1, X)
            X -= p / (nlat * (X * p - p1) / (X * X - 1))
        p = _legendre_decimal(nlat, X)
        p1 = _legendre_decimal(nlat - 1, X)
        dp = nlat * (X * p - p1) / (X * X - 1)
        W = 2 / ((1 - X * X) * dp * dp)
        assert abs(float((Decimal(float(w[j])) - W) / W)) < 1.2e-16, j


# --------------------------------------------------------------------------
# Normalised associated Legendre functions
# --------------------------------------------------------------------------

def test_legendre_closed_forms():
    o = _orc()
    xs = np.array([0.93, 0.41, 0.0, -0.27, -0.88])
    s = np.sqrt((1 - xs) * (1 + xs))
    closed = {
        (0, 0): np.ones_like(xs),
        (1, 0): math.sqrt(3) * xs,
        (1, 1): math.sqrt(1.5) * s,
        (2, 0): math.sqrt(5) / 2 * (3 * xs ** 2 - 1),
        (2, 1): math.sqrt(7.5) * xs * s,
        (2, 2): math.sqrt(15 / 8) * s ** 2,
        (3, 0): math.sqrt(7) / 2 * (5 * xs ** 3 - 3 * xs),
        (3, 1): math.sqrt(21) / 4 * s * (5 * xs ** 2 - 1),
        (3, 2): math.sqrt(105 / 8) * xs * s ** 2,
        (3, 3): math.sqrt(35) / 4 * s ** 3,
    }
    for m in range(4):
        tab = o.legendre(3, m, xs)
        for n in range(m, 4):
            assert np.allclose(tab[:, n - m], closed[(n, m)], rtol=0, atol=5e-16), (n, m)


def test_legendre_endpoints_and_parity():
    o = _orc()
    N = 200
    for m in (0, 1, 5, 77):
        at1 = o.legendre(N, m, [1.0, -1.0])
        n = np.arange(m, N + 1)
        if m == 0:
            assert np.allclose(at1[0], np.sqrt(2 * n + 1), rtol=1e-13, atol=0)
            assert np.allclose(at1[1], (-1.0) ** n * np.sqrt(2 * n + 1), rtol=1e-13, atol=0)
        else:
            assert np.all(at1 == 0.0)
    xs = np.array([0.1, 0.57, 0.999])
    for m in (0, 3, 64):
        pp = o.legendre(N, m, xs)
        pm = o.legendre(N, m, -xs)
        sign = (-1.0) ** (np.arange(m, N + 1) - m)
        assert np.array_equal(pm, pp * sign)


def test_legendre_vs_scipy_sph_harm():
    """P̄_n^m(cos t) e^{i m p} = (-1)^m sqrt(4 pi) Y_n^m(t, p) (scipy's Y carries
    the Condon-Shortley phase; P̄ does not)."""
    sp = pytest.importorskip("scipy.special")
    o = _orc()
    N = 40
    theta = np.array([0.05, 0.7, 1.3, 2.2, 3.0])
    for m in (0, 1, 2, 7, 20, 40):
        tab = o.legendre(N, m, np.cos(theta))
        for n in range(m, N + 1):
            y = sp.sph_harm_y(n, m, theta, 0.0).real
            ref = (-1.0) ** m * math.sqrt(4 * math.pi) * y
            assert np.allclose(tab[:, n - m], ref, rtol=1e-12, atol=1e-13), (n, m)


def test_legendre_discrete_orthonormality():
    """(1/2) sum_j w_j P̄_n^m P̄_n'^m = delta_nn' on nlat >= N + 1 Gauss nodes."""
    o = _orc()
    N, nlat = 63, 64
    mu, w = o.gauss(nlat)
    for m in (0, 1, 10, 40, 63):
        P = o.legendre(N, m, mu)
        G = 0.5 * (P.T * w) @ P
        assert np.max(np.abs(G - np.eye(N - m + 1))) < 2e-13, m


def test_legendre_addition_theorem_high_degree():
    """P̄_n^0^2 + 2 sum_{m>=1} (P̄_n^m)^2 = 2n + 1 at n = 1279."""
    o = _orc()
    N = 1279
    for x in (0.9995, 0.7, 0.2, -0.35):
        tot = o.legendre(N, 0, [x])[0] ** 2
        for m in range(1, N + 1):
            col = o.legendre(N, m, [x])[0]
            tot[m:] += 2 * col ** 2
        n = np.arange(N + 1)
        assert np.max(np.abs(tot / (2 * n + 1) - 1)) < 1e-10, x


def test_legendre_addition_theorem_beyond_double_range():
    """The addition theorem at every n <= 1999 (TCo1999) at points where, for
    some m, the sectoral value P̄_m^m lies far below the double range while
    P̄_n^m at higher n is of order one: a seed that underflows to zero would
    drop those terms (squares up to about 25) from the sum."""
    o = _orc()
    N = 1999
    mu2000, _ = o.gauss(4000)
    # 0.95, 0.9 and node 600 of O2000 (mu = 0.8908) lose terms up to 5.0,
    # 4.6 and 3.2 with an underflowing seed
    for x in (0.95, 0.9, float(mu2000[600])):
        s = np.sqrt((1 - x) * (1 + x))
        # log10 of P̄_m^m = prod_k sqrt((2k+1)/(2k)) s, in closed form
        k = np.arange(1, N + 1)
        log_pmm = np.concatenate([[0.0], np.cumsum(0.5 * np.log10((2 * k + 1) / (2 * k)) + np.log10(s))])
        tot = o.legendre(N, 0, [x])[0] ** 2
        lost = 0.0
        for m in range(1, N + 1):
            col = o.legendre(N, m, [x])[0]
            tot[m:] += 2 * col ** 2
            if log_pmm[m] < -310:
                lost = max(lost, float(np.max(np.abs(col))))
        n = np.arange(N + 1)
        assert np.max(np.abs(tot / (2 * n + 1) - 1)) < 1e-10, x
        # the point exercises the extended range: columns whose seed is below
        # 1e-310 still reach values above 1
        assert lost > 1.0, (x, lost)


# --------------------------------------------------------------------------
# Ring DFTs
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [20, 24, 36, 320, 1036, 5132])
def test_ring_dft_vs_numpy(n):
    o = _orc()
    rng = np.random.default_rng(n)
    g = rng.standard_normal(n)
    M = o.ring_cutoff(n, n)
    G = o.ring_dft(n, M, g)
    ref = np.fft.rfft(g)[: M + 1]
    assert np.max(np.abs(G - ref)) < 1e-12 * np.sqrt(n) * np.abs(ref).max()


@pytest.mark.parametrize("n", [20, 44, 320, 1036])
def test_ring_synth_vs_numpy(n):
    o = _orc()
    rng = np.random.default_rng(n + 1)
    M = (n - 1) // 2
    F = rng.standard_normal(M + 1) + 1j * rng.standard_normal(M + 1)
    g = o.ring_synth(n, M, F, 2.0)
    X = np.zeros(n // 2 + 1, complex)
    X[: M + 1] = F
    X[0] = F[0].real
    ref = np.fft.irfft(X, n) * n
    assert np.max(np.abs(g - ref)) < 1e-12 * np.abs(ref).max()
    # single modes: cos(m lambda) has G_m = n/2 (m >= 1)
    k = np.arange(n)
    for m in (1, 3, M):
        G = o.ring_dft(n, M, np.cos(2 * np.pi * m * k / n))
        assert abs(G[m] - n / 2) < 1e-12 * n
        G[m] = 0
        assert np.max(np.abs(G)) < 1e-12 * n


# --------------------------------------------------------------------------
# Whole transforms
# --------------------------------------------------------------------------

def _grid_coords(nlon, o):
    mu, w = o.gauss(len(nlon))
    lam = [2 * np.pi * np.arange(n) / n for n in nlon]
    return mu, w, lam


@pytest.mark.parametrize("grid", ["full", "oct"])
def test_single_harmonic(grid):
    """a_n^m = 1 gives c_m P̄_n^m(mu_j) cos(m lambda_k); a_n^m = i gives -c_m P̄ sin,
    and zero on rings whose cutoff is below m."""
    o = _orc()
    N = 23
    nlon = o.full_nlon(24, 48) if grid == "full" else o.octahedral_nlon(12)
    mu, _, lam = _grid_coords(nlon, o)
    ns = o.nspec(N)
    mm, nn = si.spec_mn(N)
    for (m, n) in [(0, 0), (0, 5), (1, 1), (3, 8), (9, 9), (12, 23)]:
        slot = int(np.flatnonzero((mm == m) & (nn == n))[0])
        for val in (1.0, 1j):
            a = np.zeros(ns, complex)
            a[slot] = val
            g = o.inv(N, nlon, a)[0]
            c = 1.0 if m == 0 else 2.0
            pos = 0
            for j, L in enumerate(nlon):
                Mj = o.ring_cutoff(N, L)
                p = o.legendre(N, m, [mu[j]])[0, n - m]
                if Mj < m:
                    ref = np.zeros(L)
                elif val == 1.0:
                    ref = c * p * np.cos(m * lam[j])
                else:
                    ref = -c * p * np.sin(m * lam[j]) if m > 0 else np.zeros(L)
                assert np.allclose(g[pos:pos + L], ref, rtol=0, atol=1e-13), (m, n, val, j)
                pos += L


def test_brute_force_series_scipy():
    """Pointwise series with scipy's Y_n^m on a small O-grid, honouring the cutoff."""
    sp = pytest.importorskip("scipy.special")
    o = _orc()
    N = 15
    nlon = o.octahedral_nlon(8)
    mu, _, lam = _grid_coords(nlon, o)
    a = si.spectral_fields(N, 99, [0])[0]
    g = o.inv(N, nlon, a)[0]
    mm, nn = si.spec_mn(N)
    theta = np.arccos(mu)
    pos = 0
    for j, L in enumerate(nlon):
        Mj = o.ring_cutoff(N, L)
        ref = np.zeros(L)
        for slot in range(len(a)):
            m, n = int(mm[slot]), int(nn[slot])
            if m > Mj:
                continue
            y = sp.sph_harm_y(n, m, theta[j], lam[j])
            ybar = (-1.0) ** m * math.sqrt(4 * math.pi) * y
            c = 1.0 if m == 0 else 2.0
            coef = a[slot] if m > 0 else a[slot].real
            ref += c * (coef * ybar).real
        assert np.allclose(g[pos:pos + L], ref, rtol=0, atol=2e-14 * np.abs(ref).max() + 1e-15), j
        pos += L


def test_round_trip_full_grid_t79():
    """T79 on the full 160 x 320 Gaussian grid: dir(inv(a)) = a (quadrature exact
    to degree 2 nlat - 1 >= 2N and no aliasing with nlon >= 2N + 1)."""
    o = _orc()
    w = si.WORKLOADS["t79_full"]
    nlon = w.ring_lengths()
    a = si.spectral_fields(w.trunc, w.key, [0])
    b = o.dir(w.trunc, nlon, o.inv(w.trunc, nlon, a))
    assert np.max(np.abs(b - a)) / np.max(np.abs(a)) < 1e-13


def test_round_trip_octahedral_defect():
    """On an O-grid dir(inv(a)) = a - E a with E_m = 1/2 sum_{j: M_j < m} w_j
    P̄^m(mu_j) P̄^m(mu_j)^T: the polar rings that cannot carry m."""
    o = _orc()
    N, nl = 31, 32
    nlon = o.octahedral_nlon(nl)
    mu, w = o.gauss(2 * nl)
    a = si.spectral_fields(N, 98, [0])[0]
    b = o.dir(N, nlon, o.inv(N, nlon, a))[0]
    mm, _ = si.spec_mn(N)
    pred = a.copy()
    for m in range(N + 1):
        rings = [j for j in range(2 * nl) if o.ring_cutoff(N, nlon[j]) < m]
        if not rings:
            continue
        P = o.legendre(N, m, mu[rings])
        E = 0.5 * (P.T * w[rings]) @ P
        sl = mm == m
        pred[sl] = a[sl] - E @ a[sl]
    assert np.max(np.abs(b - pred)) / np.max(np.abs(a)) < 1e-14
    assert np.max(np.abs(b - a)) / np.max(np.abs(a)) < 1e-12


def test_parseval_full_grid():
    o = _orc()
    N = 31
    nlon = o.full_nlon(32, 64)
    _, w = o.gauss(32)
    a = si.spectral_fields(N, 97, [0])[0]
    g = o.inv(N, nlon, a)[0].reshape(32, 64)
    lhs = 0.5 * np.sum(w[:, None] / 64 * g ** 2)
    mm, _ = si.spec_mn(N)
    rhs = np.sum(np.abs(a[mm == 0].real) ** 2) + 2 * np.sum(np.abs(a[mm > 0]) ** 2)
    assert abs(lhs - rhs) / rhs < 1e-14


def _rdot_spec(a, b):
    return float(np.sum(a.real * b.real + a.imag * b.imag))


@pytest.mark.parametrize("N,grid", [(7, "oct"), (15, "full"), (31, "oct")])
def test_adjoint_dot_products(N, grid):
    o = _orc()
    nlon = o.octahedral_nlon(N + 1) if grid == "oct" else o.full_nlon(N + 1, 2 * N + 2)
    npts = int(nlon.sum())
    mm, _ = si.spec_mn(N)
    a = si.spectral_fields(N, 96, [0])[0]
    b = si.spectral_fields(N, 95, [0])[0]
    b[mm == 0] = b[mm == 0].real  # Im b_n^0 is not part of the space
    y = si.white_noise_grid(npts, 94)
    lhs = float(np.dot(o.inv(N, nlon, a)[0], y))
    rhs = _rdot_spec(a, o.inv_adj(N, nlon, y)[0])
    assert abs(lhs - rhs) <= 1e-14 * (abs(lhs) + np.linalg.norm(y) * np.linalg.norm(a))
    lhs = _rdot_spec(o.dir(N, nlon, y)[0], b)
    rhs = float(np.dot(y, o.dir_adj(N, nlon, b)[0]))
    assert abs(lhs - rhs) <= 1e-14 * (abs(lhs) + np.linalg.norm(y) * np.linalg.norm(b))


def test_inv_adj_is_weighted_direct():
    """inv_adj(y) = c_m dir(h) with h_{j,k} = 2 nlon_j y_{j,k} / w_j."""
    o = _orc()
    N, nl = 15, 16
    nlon = o.octahedral_nlon(nl)
    _, w = o.gauss(2 * nl)
    y = si.white_noise_grid(int(nlon.sum()), 93)
    scale = np.concatenate([np.full(L, 2 * L / w[j]) for j, L in enumerate(nlon)])
    d = o.dir(N, nlon, y * scale)[0]
    mm, _ = si.spec_mn(N)
    d = d * np.where(mm == 0, 1.0, 2.0)
    assert np.max(np.abs(o.inv_adj(N, nlon, y)[0] - d)) < 1e-12 * np.abs(d).max()


def test_imaginary_part_at_m0_ignored():
    o = _orc()
    N = 15
    nlon = o.octahedral_nlon(16)
    a = si.spectral_fields(N, 92, [0])[0]
    mm, _ = si.spec_mn(N)
    b = a.copy()
    b[mm == 0] += 1j * 3.0
    assert np.array_equal(o.inv(N, nlon, a), o.inv(N, nlon, b))
    assert np.array_equal(o.dir_adj(N, nlon, a), o.dir_adj(N, nlon, b))
    d = o.dir(N, nlon, o.inv(N, nlon, a))[0]
    assert np.all(d[mm == 0].imag == 0)


def test_workload_geometry():
    """Ring lengths and maxima of the five workload grids."""
    o = _orc()
    for key, mx in [("t255_o256", 1040), ("tco639_o640", 2576), ("t399_o400", 1616),
                    ("tco1279_o1280", 5136)]:
        w = si.WORKLOADS[key]
        nl = w.ring_lengths()
        assert np.array_equal(nl, o.octahedral_nlon(w.nlat // 2))
        assert nl.max() == mx and nl[0] == 20 and nl[-1] == 20
    w = si.WORKLOADS["tco1279_o1280"]
    assert int(w.ring_lengths().sum()) == 6599680


# --------------------------------------------------------------------------
# Wind images from vorticity and divergence
# --------------------------------------------------------------------------

def test_legendre_deriv_vs_finite_differences():
    """H_n^m = (1 - mu^2) dP̄_n^m/dmu against a fourth-order central difference
    of the oracle's own P̄ columns."""
    o = _orc()
    N, h = 40, 1e-4
    for m in (0, 1, 7, 25):
        for x in (-0.83, 0.05, 0.61):
            H = o.legendre_deriv(N, m, x)
            P = [o.legendre(N, m, [x + k * h])[0] for k in (-2, -1, 1, 2)]
            dP = (P[0] - 8 * P[1] + 8 * P[2] - P[3]) / (12 * h)
            assert np.max(np.abs(H - (1 - x * x) * dP)) < 1e-8 * max(1.0, np.abs(H).max()), (m, x)


def _uv_closed_form_grid(N, nlon, which):
    o = _orc()
    mu, _ = o.gauss(len(nlon))
    ns = o.nspec(N)
    z = np.zeros((1, ns), complex)
    d = np.zeros((1, ns), complex)
    idx = {(0, 1): 1, (1, 1): N + 1}  # m-major index of (m, n) = (0, 1) and (1, 1)
    lam, mus = [], []
    for j, n in enumerate(nlon):
        lam.append(2 * np.pi * np.arange(n) / n)
        mus.append(np.full(n, mu[j]))
    lam, x = np.concatenate(lam), np.concatenate(mus)
    s = np.sqrt((1 - x) * (1 + x))
    c = np.sqrt(1.5)
    if which == "rotation":      # zeta_1^0 = 2: U = sqrt(3) (1 - mu^2), V = 0
        z[0, idx[(0, 1)]] = 2.0
        U, V = np.sqrt(3) * (1 - x * x), 0 * x
    elif which == "vortex11":    # zeta_1^1 = 1
        z[0, idx[(1, 1)]] = 1.0
        U, V = -c * x * s * np.cos(lam), c * s * np.sin(lam)
    else:                        # D_1^1 = 1
        d[0, idx[(1, 1)]] = 1.0
        U, V = c * s * np.sin(lam), c * x * s * np.cos(lam)
    return o.uv(N, nlon, z, d), U, V


@pytest.mark.parametrize("which", ["rotation", "vortex11", "divergent11"])
def test_uv_closed_forms(which):
    """Solid-body rotation and the m = 1 vortex and source: U = u cos(phi) and
    V = v cos(phi) in closed form, on an octahedral grid with cutoff."""
    o = _orc()
    nlon = o.octahedral_nlon(16)
    g, U, V = _uv_closed_form_grid(15, nlon, which)
    assert np.max(np.abs(g[0] - U)) < 1e-13
    assert np.max(np.abs(g[1] - V)) < 1e-13


def test_uv_kinetic_energy():
    """Full Gaussian grid, random band-limited vorticity and divergence: the
    quadrature of u^2 + v^2 = (U^2 + V^2) / (1 - mu^2) equals
    sum_{n >= 1} c_m n (n + 1) (|psi_n^m|^2 + |chi_n^m|^2) (exact: the
    lambda-mean of u^2 + v^2 is a polynomial of degree 2N in mu)."""
    import synth_inputs as si
    o = _orc()
    N, nlat, nl = 31, 64, 128
    nlon = o.full_nlon(nlat, nl)
    mu, w = o.gauss(nlat)
    zeta = si.spectral_fields(N, 91, [0, 1])
    dvg = si.spectral_fields(N, 92, [0, 1])
    g = o.uv(N, nlon, zeta, dvg)
    m, n = si.spec_mn(N)
    cm = np.where(m == 0, 1.0, 2.0)
    lap = np.where(n > 0, -1.0 / np.maximum(n * (n + 1), 1), 0.0)
    for f in range(2):
        psi, chi = zeta[f] * lap, dvg[f] * lap
        psi = np.where(m == 0, psi.real, psi)
        chi = np.where(m == 0, chi.real, chi)
        rhs = np.sum(cm * n * (n + 1) * (np.abs(psi) ** 2 + np.abs(chi) ** 2))
        U, V = g[f].reshape(nlat, nl), g[2 + f].reshape(nlat, nl)
        lhs = 0.5 * np.sum(w[:, None] / nl * (U ** 2 + V ** 2) / (1 - mu[:, None] ** 2))
        assert abs(lhs - rhs) < 1e-13 * rhs, (f, lhs, rhs)
