"""Error metrics for comparing transform outputs with the FP64 oracle (used by
the tests and the benchmark; no transform arithmetic).

Spectral: e_max = max|a_hat - a| / max|a|, e_rms = sqrt(sum c_m |a_hat - a|^2 /
sum c_m |a|^2) with c_0 = 1, c_m = 2 (the area-weighted grid RMS by Parseval).
Grid: e_max = max|g_hat - g| / max|g|, e_rms weighted by w_j / nlon_j.
All per field; callers take the max over fields.
"""
import numpy as np

import synth_inputs as si


def spec_errors(a_hat, a, trunc):
    a_hat = np.atleast_2d(np.asarray(a_hat, dtype=np.complex128))
    a = np.atleast_2d(np.asarray(a, dtype=np.complex128))
    m, _ = si.spec_mn(trunc)
    c = np.where(m == 0, 1.0, 2.0)
    d = a_hat - a
    e_max = np.abs(d).max(axis=1) / np.abs(a).max(axis=1)
    e_rms = np.sqrt((c * np.abs(d) ** 2).sum(axis=1) / (c * np.abs(a) ** 2).sum(axis=1))
    return e_max, e_rms


def grid_errors(g_hat, g, nlon, w):
    g_hat = np.atleast_2d(np.asarray(g_hat, dtype=np.float64))
    g = np.atleast_2d(np.asarray(g, dtype=np.float64))
    wt = np.concatenate([np.full(int(n), wj / n) for n, wj in zip(nlon, w)])
    d = g_hat - g
    e_max = np.abs(d).max(axis=1) / np.abs(g).max(axis=1)
    e_rms = np.sqrt((wt * d ** 2).sum(axis=1) / (wt * g ** 2).sum(axis=1))
    return e_max, e_rms
