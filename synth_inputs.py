"""Seeded synthetic inputs and workload descriptions.

This module is shared by the tests, the smoke check and the benchmark, and
feeds both the HIP path and the CPU oracle.  It holds no transform
arithmetic: only the workload shapes and the random-number recipe.

Recipe for field ``f`` of workload ``K``: a PCG64 generator seeded with
``1000 * K + f`` draws ``re`` then ``im`` as ``nspec`` standard normals each,
in m-major order (m = 0..N, n = m..N); the coefficient is
``(re + i im) * (n + 1) ** -1.5`` and the imaginary part is zero for m = 0.
Band-limited grids for direct-only tests are made by the caller from these
coefficients; white-noise grids use the same seeding with standard normals.
"""
import functools
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Workload:
    key: int          # seed block (1000 * key + field)
    name: str
    trunc: int        # triangular truncation N
    grid: str         # "full" or "octahedral"
    nlat: int         # number of Gaussian latitudes
    nlon_full: int    # ring length of a full grid (0 for octahedral)
    nfld: int         # number of independent scalar fields
    prec: str         # Legendre arithmetic form: fp64 | fp32 | bf16x3 | fp16x3

    def ring_lengths(self) -> np.ndarray:
        """Ring lengths north to south: full grid, or O_{nlat/2} with 20 + 4 i points
        on the i-th ring from the nearer pole."""
        if self.grid == "full":
            return np.full(self.nlat, self.nlon_full, dtype=np.int32)
        nl = self.nlat // 2
        i = np.arange(self.nlat)
        i = np.where(i < nl, i, self.nlat - 1 - i)
        return (20 + 4 * i).astype(np.int32)


# The five workloads: T79 full 160x320 (1 field, FP64), T255/O256 (411 fields,
# FP32), TCo639/O640 (411, split BF16), T399/O400 (137, FP32, adjoint),
# TCo1279/O1280 (411, FP32 and split BF16); and the 5 km case the paper runs
# beyond them, TCo1999/O2000 (4000 latitudes, rings up to 8016 points; 411
# fields, FP32).
WORKLOADS = {
    "t79_full": Workload(1, "T79 full Gaussian 160x320", 79, "full", 160, 320, 1, "fp64"),
    "t255_o256": Workload(2, "T255 O256", 255, "octahedral", 512, 0, 411, "fp32"),
    "tco639_o640": Workload(3, "TCo639 O640", 639, "octahedral", 1280, 0, 411, "bf16x3"),
    "t399_o400": Workload(4, "T399 O400", 399, "octahedral", 800, 0, 137, "fp32"),
    "tco1279_o1280": Workload(5, "TCo1279 O1280", 1279, "octahedral", 2560, 0, 411, "fp32"),
    "tco1999_o2000": Workload(6, "TCo1999 O2000", 1999, "octahedral", 4000, 0, 411, "fp32"),
}


def nspec(trunc: int) -> int:
    return (trunc + 1) * (trunc + 2) // 2


@functools.lru_cache(maxsize=8)
def spec_mn(trunc: int):
    """(m, n) of every m-major spectral slot (read-only arrays, cached)."""
    m = np.concatenate([np.full(trunc + 1 - mm, mm) for mm in range(trunc + 1)])
    n = np.concatenate([np.arange(mm, trunc + 1) for mm in range(trunc + 1)])
    m.flags.writeable = False
    n.flags.writeable = False
    return m, n


@functools.lru_cache(maxsize=8)
def _spectrum(trunc: int):
    """(n + 1)^-1.5 per slot and the number of m = 0 slots (they come first)."""
    m, n = spec_mn(trunc)
    sc = (n + 1.0) ** -1.5
    sc.flags.writeable = False
    return sc, trunc + 1


def spectral_field(trunc: int, seed: int) -> np.ndarray:
    """One complex128 spectral field with the (n+1)^-1.5 spectrum."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = nspec(trunc)
    re = rng.standard_normal(ns)
    im = rng.standard_normal(ns)
    sc, n0 = _spectrum(trunc)
    im[:n0] = 0.0  # m = 0: real coefficients
    a = np.empty(ns, dtype=np.complex128)
    a.real = re * sc
    a.imag = im * sc
    return a


def spectral_fields(trunc: int, key: int, fields) -> np.ndarray:
    """[len(fields), nspec] complex128 for the given field indices of workload ``key``."""
    return np.stack([spectral_field(trunc, 1000 * key + int(f)) for f in fields])


def white_noise_grid(npts: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(npts)


def random_unit(shape, seed: int, complex_: bool = False) -> np.ndarray:
    """Seeded random direction of unit Euclidean norm (real, or complex viewed as 2 reals)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if complex_:
        v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    else:
        v = rng.standard_normal(shape)
    return v / np.sqrt(np.sum(np.abs(v) ** 2))
