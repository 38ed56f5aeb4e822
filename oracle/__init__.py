"""FP64 CPU oracle for the spherical-harmonic transform pair (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  It loads ``liboracle.so`` (plain C,
built by ``oracle/build.py``) and shares nothing with the HIP library.

The formulas it evaluates are written out in ``shtx_oracle.c``; this module
only marshals numpy arrays:

* spectral arrays are complex128 ``[nfld, nspec]``, m-major, n ascending;
* grid arrays are float64 ``[nfld, npts]``, rings north to south.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError("oracle library not built: run `python oracle/build.py` "
                           "or __graft_entry__.build()")
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_octahedral_nlon.argtypes = [ctypes.c_int, _i32p]
    lib.oracle_ring_cutoff.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.oracle_ring_cutoff.restype = ctypes.c_int
    lib.oracle_nspec.argtypes = [ctypes.c_int]
    lib.oracle_nspec.restype = ctypes.c_int64
    lib.oracle_gauss.argtypes = [ctypes.c_int, _f64p, _f64p]
    lib.oracle_legendre.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _f64p, _f64p]
    for name in ("oracle_inv", "oracle_dir", "oracle_inv_adj", "oracle_dir_adj"):
        getattr(lib, name).argtypes = [ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int,
                                       _f64p, _f64p, ctypes.c_int]
    lib.oracle_ring_synth.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _f64p, _f64p]
    lib.oracle_ring_dft.argtypes = [ctypes.c_int, ctypes.c_int, _f64p, _f64p]
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_legendre_deriv.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _f64p]
    lib.oracle_uv.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int, _f64p, _f64p, _f64p, ctypes.c_int]
    _lib = lib
    return lib


def octahedral_nlon(nl: int) -> np.ndarray:
    """Ring lengths of the octahedral grid O_nl (2 nl rings, north to south)."""
    out = np.empty(2 * nl, dtype=np.int32)
    _load().oracle_octahedral_nlon(nl, out)
    return out


def full_nlon(nlat: int, nlon: int) -> np.ndarray:
    """Ring lengths of a full (regular) Gaussian grid."""
    return np.full(nlat, nlon, dtype=np.int32)


def ring_cutoff(trunc: int, nlon: int) -> int:
    return _load().oracle_ring_cutoff(trunc, int(nlon))


def nspec(trunc: int) -> int:
    return int(_load().oracle_nspec(trunc))


def gauss(nlat: int):
    """Gauss-Legendre nodes (descending) and weights, FP64."""
    mu = np.empty(nlat)
    w = np.empty(nlat)
    _load().oracle_gauss(nlat, mu, w)
    return mu, w


def legendre(trunc: int, m: int, mu) -> np.ndarray:
    """P̄_n^m(mu_i) for n = m..trunc: array [len(mu), trunc - m + 1]."""
    mu = np.ascontiguousarray(np.atleast_1d(np.asarray(mu, dtype=np.float64)))
    out = np.empty((mu.size, trunc - m + 1))
    _load().oracle_legendre(trunc, m, mu.size, mu, out)
    return out


def _geom(nlon):
    nlon = np.ascontiguousarray(np.asarray(nlon, dtype=np.int32))
    return nlon, int(nlon.size), int(nlon.sum())


def _spec_in(spec, trunc):
    spec = np.asarray(spec)
    if spec.ndim == 1:
        spec = spec[None]
    if spec.shape[1] != nspec(trunc):
        raise ValueError(f"spectral array has {spec.shape[1]} coefficients, expected {nspec(trunc)}")
    s = np.ascontiguousarray(spec.astype(np.complex128, copy=False))
    return s.view(np.float64).reshape(s.shape[0], -1), s.shape[0]


def _grid_in(grid, npts):
    grid = np.asarray(grid, dtype=np.float64)
    if grid.ndim == 1:
        grid = grid[None]
    if grid.shape[1] != npts:
        raise ValueError(f"grid array has {grid.shape[1]} points, expected {npts}")
    return np.ascontiguousarray(grid), grid.shape[0]


def _synth(name, trunc, nlon, spec, nthreads):
    nlon, nlat, npts = _geom(nlon)
    s, nfld = _spec_in(spec, trunc)
    out = np.empty((nfld, npts))
    getattr(_load(), name)(trunc, nlat, nlon, nfld, s, out, int(nthreads))
    return out


def _anal(name, trunc, nlon, grid, nthreads):
    nlon, nlat, npts = _geom(nlon)
    g, nfld = _grid_in(grid, npts)
    out = np.empty((nfld, 2 * nspec(trunc)))
    getattr(_load(), name)(trunc, nlat, nlon, nfld, g, out, int(nthreads))
    return out.view(np.complex128)


def inv(trunc, nlon, spec, nthreads=0):
    """Inverse transform spectral -> grid."""
    return _synth("oracle_inv", trunc, nlon, spec, nthreads)


def dir(trunc, nlon, grid, nthreads=0):  # noqa: A001 - the transform's name
    """Direct transform grid -> spectral."""
    return _anal("oracle_dir", trunc, nlon, grid, nthreads)


def inv_adj(trunc, nlon, grid, nthreads=0):
    """Adjoint of the inverse transform (grid -> spectral)."""
    return _anal("oracle_inv_adj", trunc, nlon, grid, nthreads)


def dir_adj(trunc, nlon, spec, nthreads=0):
    """Adjoint of the direct transform (spectral -> grid)."""
    return _synth("oracle_dir_adj", trunc, nlon, spec, nthreads)


def ring_synth(n: int, M: int, F, fac_pos: float = 2.0) -> np.ndarray:
    """g_k = sum_{m<=M} fac_m Re(F_m e^{2 pi i m k/n}), fac_0 = 1, fac_m = fac_pos."""
    F = np.ascontiguousarray(np.asarray(F, dtype=np.complex128)[: M + 1])
    g = np.empty(n)
    _load().oracle_ring_synth(n, M, float(fac_pos), F.view(np.float64), g)
    return g


def ring_dft(n: int, M: int, g) -> np.ndarray:
    """G_m = sum_k g_k e^{-2 pi i m k/n} for m = 0..M (unscaled naive DFT)."""
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float64))
    out = np.empty(2 * (M + 1))
    _load().oracle_ring_dft(n, M, g, out)
    return out.view(np.complex128)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def legendre_deriv(trunc: int, m: int, mu: float) -> np.ndarray:
    """H_n^m(mu) = (1 - mu^2) dP̄_n^m/dmu for n = m..trunc at one abscissa."""
    out = np.empty(trunc - m + 1)
    _load().oracle_legendre_deriv(trunc, m, float(mu), out)
    return out


def uv(trunc, nlon, vor, div, nthreads=0):
    """Wind images U = u cos(phi), V = v cos(phi) on the unit sphere from
    spectral vorticity and divergence [nfld, nspec]: grid [2 nfld, npts], U of
    field f in row f, V in row nfld + f."""
    nlon, nlat, npts = _geom(nlon)
    z, nfld = _spec_in(vor, trunc)
    d, nfld2 = _spec_in(div, trunc)
    if nfld2 != nfld:
        raise ValueError("vorticity and divergence hold different field counts")
    out = np.empty((2 * nfld, npts))
    _load().oracle_uv(trunc, nlat, nlon, nfld, z, d, out, int(nthreads))
    return out
