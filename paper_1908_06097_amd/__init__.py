"""Spherical-harmonic transforms on AMD MI355X: Python binding of libshtx.

This module only marshals arguments: every step of every transform runs in
the HIP kernels of ``libshtx.so`` (built in-tree by ``build.py``).  PyTorch
provides device memory and the stream; there is no CPU fallback, and using a
transform without the built library or without a GPU raises.

The transforms, layouts and precision forms are those of ``include/shtx.h``:

* spectral arrays: ``[nfld, nspec]`` complex (complex128 for ``fp64`` plans,
  complex64 otherwise), m-major, n ascending;
* grid arrays: ``[nfld, npts]`` real (float64 / float32), rings north to
  south.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshtx.so")

GRIDS = {"full": 0, "octahedral": 1}
PRECS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16x3": 3}
FLAG_GRAPH = 1
FLAG_TIMING = 2
FLAG_AUTOTUNE = 4
FLAG_UV = 8
# shtx_probe_peak kinds: compute probes return TFLOP/s, memory probes GB/s
PROBES = {"mfma_f64": 0, "mfma_f32": 1, "mfma_bf16": 2, "mfma_f16": 3, "valu_f32": 4, "hbm_copy": 5,
          "hbm_read": 6}

_lib = None

_EXPORTS = ("shtx_plan_create", "shtx_plan_check", "shtx_plan_check_shapes", "shtx_plan_set_shapes", "shtx_plan_info", "shtx_plan_ring_lengths", "shtx_plan_nodes",
            "shtx_plan_legendre", "shtx_inv_trans", "shtx_dir_trans", "shtx_inv_trans_adj",
            "shtx_dir_trans_adj", "shtx_uv_trans", "shtx_inv_trans_noalloc", "shtx_timing_reset", "shtx_timing_enable", "shtx_timing_read", "shtx_plan_destroy",
            "shtx_probe_peak", "shtx_strerror")


class ShtxError(RuntimeError):
    pass


class Info(ctypes.Structure):
    _fields_ = [("trunc", ctypes.c_int32), ("nlat", ctypes.c_int32), ("nfld", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("grid", ctypes.c_int32), ("max_nlon", ctypes.c_int32),
                ("nspec", ctypes.c_int64), ("npts", ctypes.c_int64), ("nfour", ctypes.c_int64),
                ("table_bytes", ctypes.c_size_t), ("workspace_bytes", ctypes.c_size_t),
                ("legendre_flops", ctypes.c_double), ("plan_seconds", ctypes.c_double),
                ("inv_tile", ctypes.c_int32 * 2), ("dir_tile", ctypes.c_int32 * 2), ("fft_cap", ctypes.c_int32),
                ("tuned", ctypes.c_int32)]


def load_library():
    """Load libshtx.so and declare its C signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ShtxError(f"HIP library missing: {LIB_PATH} (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, u32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint
    lib.shtx_plan_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, i32, i32, i32, u32, vp]
    lib.shtx_plan_info.argtypes = [vp, ctypes.POINTER(Info)]
    lib.shtx_plan_check.argtypes = [i32, i32, i32, i32, i32, i32, ctypes.POINTER(Info)]
    lib.shtx_plan_check_shapes.argtypes = [i32] * 11 + [ctypes.POINTER(Info)]
    lib.shtx_plan_set_shapes.argtypes = [vp] + [i32] * 5
    lib.shtx_plan_ring_lengths.argtypes = [vp, ctypes.c_void_p]
    lib.shtx_plan_nodes.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p]
    lib.shtx_plan_legendre.argtypes = [vp, i32, ctypes.c_void_p]
    for name in ("shtx_inv_trans", "shtx_dir_trans", "shtx_inv_trans_adj", "shtx_dir_trans_adj",
                 "shtx_inv_trans_noalloc"):
        getattr(lib, name).argtypes = [vp, vp, vp, vp]
    lib.shtx_uv_trans.argtypes = [vp, vp, vp, vp, vp]
    lib.shtx_timing_reset.argtypes = [vp]
    lib.shtx_timing_enable.argtypes = [vp, i32]
    lib.shtx_timing_read.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p]
    lib.shtx_plan_destroy.argtypes = [vp]
    lib.shtx_probe_peak.argtypes = [i32, vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double), vp]
    lib.shtx_strerror.argtypes = [i32]
    lib.shtx_strerror.restype = ctypes.c_char_p
    for name in _EXPORTS:
        if name not in ("shtx_strerror",):
            getattr(lib, name).restype = i32
    _lib = lib
    return lib


def probe_peak(kind, src=None, dst=None):
    """Rate one peak probe measures on torch's current device and stream
    (shtx_probe_peak): TFLOP/s for "mfma_f64", "mfma_f32", "mfma_bf16",
    "mfma_f16", "valu_f32"; GB/s for "hbm_copy" (src -> dst, both counted)
    and "hbm_read" (src).  src/dst: contiguous device tensors of the same
    byte size (a multiple of 16, at least 1 MiB) for the memory probes."""
    import torch
    if kind not in PROBES:
        raise ShtxError(f"unknown probe {kind!r}; expected one of {sorted(PROBES)}")
    if not torch.cuda.is_available():
        raise ShtxError("libshtx needs a ROCm GPU; no CPU fallback exists")
    nbytes = 0
    if kind in ("hbm_copy", "hbm_read"):
        if src is None or not src.is_cuda or not src.is_contiguous():
            raise ShtxError("memory probes need a contiguous device tensor src")
        nbytes = src.numel() * src.element_size()
        if kind == "hbm_copy" and (dst is None or not dst.is_cuda or not dst.is_contiguous()
                                   or dst.numel() * dst.element_size() < nbytes):
            raise ShtxError("the copy probe needs a contiguous device tensor dst at least as large as src")
    if dst is None:
        dst = torch.empty(4, dtype=torch.float32, device=src.device if src is not None else "cuda")
    rate = ctypes.c_double(0.0)
    stream = torch.cuda.current_stream(dst.device).cuda_stream
    _check(load_library().shtx_probe_peak(PROBES[kind], ctypes.c_void_p(src.data_ptr() if src is not None else 0),
                                          ctypes.c_void_p(dst.data_ptr()), ctypes.c_size_t(nbytes),
                                          ctypes.byref(rate), ctypes.c_void_p(stream)), "shtx_probe_peak")
    return rate.value


def plan_check(trunc, grid="octahedral", nlat=None, nfld=1, prec="fp32", nlon_full=0):
    """Host-only dry run of plan creation (no GPU): returns (status, Info)."""
    lib = load_library()
    if nlat is None:
        nlat = 2 * (trunc + 1)
    info = Info()
    rc = lib.shtx_plan_check(trunc, GRIDS[grid], nlat, nlon_full, nfld, PRECS[prec], ctypes.byref(info))
    return rc, info


def plan_check_shapes(trunc, grid, nlat, nfld, prec, inv_tile, dir_tile, fft_cap, nlon_full=0):
    """Host-only dry run with explicit GEMM tile shapes and FFT blocking."""
    lib = load_library()
    info = Info()
    rc = lib.shtx_plan_check_shapes(trunc, GRIDS[grid], nlat, nlon_full, nfld, PRECS[prec], inv_tile[0],
                                    inv_tile[1], dir_tile[0], dir_tile[1], fft_cap, ctypes.byref(info))
    return rc, info


def _check(rc, what):
    if rc < 0:
        raise ShtxError(f"{what} failed: {load_library().shtx_strerror(rc).decode()} ({rc})")
    return rc


class Plan:
    """A transform plan: tables and workspace for (trunc, grid, nfld, prec) on
    the current CUDA/HIP device.  Transforms run on torch's current stream."""

    def __init__(self, trunc, grid="octahedral", nlat=None, nfld=1, prec="fp32", nlon_full=0,
                 graph=False, timing=False, autotune=False, uv=False):
        import torch
        if not torch.cuda.is_available():
            raise ShtxError("libshtx needs a ROCm GPU; no CPU fallback exists")
        lib = load_library()
        if nlat is None:
            nlat = 2 * (trunc + 1)
        self.trunc, self.grid, self.nlat, self.nfld, self.prec = trunc, grid, nlat, nfld, prec
        flags = ((FLAG_GRAPH if graph else 0) | (FLAG_TIMING if timing else 0) | (FLAG_AUTOTUNE if autotune else 0)
                 | (FLAG_UV if uv else 0))
        h = ctypes.c_void_p()
        stream = torch.cuda.current_stream().cuda_stream
        _check(lib.shtx_plan_create(ctypes.byref(h), trunc, GRIDS[grid], nlat, nlon_full, nfld,
                                    PRECS[prec], flags, ctypes.c_void_p(stream)), "shtx_plan_create")
        self._h = h
        self.info = Info()
        _check(lib.shtx_plan_info(h, ctypes.byref(self.info)), "shtx_plan_info")
        self.nspec = int(self.info.nspec)
        self.npts = int(self.info.npts)
        self.real_dtype = torch.float64 if prec == "fp64" else torch.float32
        self.complex_dtype = torch.complex128 if prec == "fp64" else torch.complex64

    def set_shapes(self, inv_tile, dir_tile, fft_cap):
        """Pin the GEMM tile shapes and FFT blocking (see shtx_plan_set_shapes)."""
        _check(load_library().shtx_plan_set_shapes(self._h, inv_tile[0], inv_tile[1], dir_tile[0], dir_tile[1],
                                                   fft_cap), "shtx_plan_set_shapes")
        _check(load_library().shtx_plan_info(self._h, ctypes.byref(self.info)), "shtx_plan_info")

    # -- geometry and tables --------------------------------------------------
    def ring_lengths(self):
        out = np.empty(self.nlat, dtype=np.int32)
        _check(load_library().shtx_plan_ring_lengths(self._h, out.ctypes.data), "ring_lengths")
        return out

    def nodes(self):
        mu = np.empty(self.nlat)
        w = np.empty(self.nlat)
        _check(load_library().shtx_plan_nodes(self._h, mu.ctypes.data, w.ctypes.data), "nodes")
        return mu, w

    def legendre(self, m):
        """Stored P̄_n^m table for wavenumber m as [R_m, trunc - m + 1] float64,
        and the first northern ring index it covers."""
        lib = load_library()
        R = _check(lib.shtx_plan_legendre(self._h, m, None), "legendre")
        out = np.zeros((R, self.trunc - m + 1))
        if R:
            _check(lib.shtx_plan_legendre(self._h, m, out.ctypes.data), "legendre")
        return out

    # -- transforms -----------------------------------------------------------
    def _prep(self, x, kind):
        import torch
        if not x.is_cuda:
            raise ShtxError("transform inputs must be device tensors")
        if kind == "spec":
            if x.dtype != self.complex_dtype or tuple(x.shape) != (self.nfld, self.nspec):
                raise ShtxError(f"spectral input must be {self.complex_dtype} [{self.nfld}, {self.nspec}],"
                                f" got {x.dtype} {tuple(x.shape)}")
        else:
            if x.dtype != self.real_dtype or tuple(x.shape) != (self.nfld, self.npts):
                raise ShtxError(f"grid input must be {self.real_dtype} [{self.nfld}, {self.npts}],"
                                f" got {x.dtype} {tuple(x.shape)}")
        return x.contiguous()

    def _out(self, kind, out, device):
        import torch
        if kind == "spec":
            shape, dt = (self.nfld, self.nspec), self.complex_dtype
        else:
            shape, dt = (self.nfld, self.npts), self.real_dtype
        if out is None:
            return torch.empty(shape, dtype=dt, device=device)
        if not out.is_cuda or out.device != device:
            raise ShtxError(f"output must be a device tensor on {device}, got {out.device}")
        if out.dtype != dt or tuple(out.shape) != shape or not out.is_contiguous():
            raise ShtxError(f"output must be a contiguous {dt} {list(shape)} tensor, got {out.dtype} "
                            f"{list(out.shape)}")
        return out

    def _run(self, fn, x, kind_in, kind_out, out):
        import torch
        x = self._prep(x, kind_in)
        y = self._out(kind_out, out, x.device)
        stream = torch.cuda.current_stream(x.device).cuda_stream
        _check(getattr(load_library(), fn)(self._h, ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(stream)), fn)
        return y

    def inv(self, spec, out=None):
        """Inverse transform: spectral [nfld, nspec] -> grid [nfld, npts]."""
        return self._run("shtx_inv_trans", spec, "spec", "grid", out)

    def uv(self, vor, div, out=None):
        """Wind images U = u cos(phi), V = v cos(phi) from vorticity and
        divergence (plans made with uv=True: truncation N + 1, 2 F fields):
        vor, div [F, (N+1)(N+2)/2] complex -> grid [2 F, npts], U rows first."""
        import torch
        F, nsw = self.nfld // 2, self.trunc * (self.trunc + 1) // 2
        xs = []
        for x in (vor, div):
            if not x.is_cuda or x.dtype != self.complex_dtype or tuple(x.shape) != (F, nsw):
                raise ShtxError(f"wind inputs must be device {self.complex_dtype} [{F}, {nsw}], "
                                f"got {x.dtype} {tuple(x.shape)} on {x.device}")
            xs.append(x.contiguous())
        y = self._out("grid", out, xs[0].device)
        stream = torch.cuda.current_stream(xs[0].device).cuda_stream
        _check(load_library().shtx_uv_trans(self._h, ctypes.c_void_p(xs[0].data_ptr()),
                                            ctypes.c_void_p(xs[1].data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                            ctypes.c_void_p(stream)), "shtx_uv_trans")
        return y

    def inv_noalloc(self, spec, out):
        """Inverse transform through shtx_inv_trans_noalloc: the library's static
        scratch instead of the plan's workspace (`out` is required, so that
        the call allocates nothing)."""
        return self._run("shtx_inv_trans_noalloc", spec, "spec", "grid", out)

    def dir(self, grid, out=None):  # noqa: A003 - the transform's name
        """Direct transform: grid [nfld, npts] -> spectral [nfld, nspec]."""
        return self._run("shtx_dir_trans", grid, "grid", "spec", out)

    def inv_adj(self, grid, out=None):
        """Adjoint of the inverse transform: grid -> spectral."""
        return self._run("shtx_inv_trans_adj", grid, "grid", "spec", out)

    def dir_adj(self, spec, out=None):
        """Adjoint of the direct transform: spectral -> grid."""
        return self._run("shtx_dir_trans_adj", spec, "spec", "grid", out)

    # -- timing -------------------------------------------------------------------
    def timing_reset(self):
        _check(load_library().shtx_timing_reset(self._h), "timing_reset")

    def timing_enable(self, on=True):
        """Per-kernel event timing on or off (plans made with timing=True)."""
        _check(load_library().shtx_timing_enable(self._h, 1 if on else 0), "timing_enable")

    def timing_read(self):
        """Summed kernel milliseconds and launch counts: [inv GEMM, dir GEMM, c2r, r2c]."""
        ms = np.zeros(4)
        cnt = np.zeros(4, dtype=np.int32)
        _check(load_library().shtx_timing_read(self._h, ms.ctypes.data, cnt.ctypes.data), "timing_read")
        return ms, cnt

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().shtx_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd():
    import torch

    class InvTrans(torch.autograd.Function):
        """grid = inv(spec); backward applies the hand-written inv_trans_adj."""

        @staticmethod
        def forward(ctx, spec, plan):
            ctx.plan = plan
            return plan.inv(spec)

        @staticmethod
        def backward(ctx, grad_grid):
            return ctx.plan.inv_adj(grad_grid.contiguous()), None

    class DirTrans(torch.autograd.Function):
        """spec = dir(grid); backward applies the hand-written dir_trans_adj."""

        @staticmethod
        def forward(ctx, grid, plan):
            ctx.plan = plan
            return plan.dir(grid)

        @staticmethod
        def backward(ctx, grad_spec):
            return ctx.plan.dir_adj(grad_spec.contiguous()), None

    return InvTrans, DirTrans


def __getattr__(name):
    if name in ("InvTrans", "DirTrans"):
        inv_t, dir_t = _autograd()
        globals()["InvTrans"], globals()["DirTrans"] = inv_t, dir_t
        return globals()[name]
    raise AttributeError(name)
