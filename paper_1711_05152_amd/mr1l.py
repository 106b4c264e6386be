"""Python binding of the multiple rank-1 lattice FFT (same names as the C ABI in include/mr1l.h).

PyTorch only supplies device memory and the current HIP stream; every step of the transform runs
in libmr1l's kernels.  There is no CPU path: without a built library or a GPU these calls raise.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import check, lib

__all__ = ["Plan", "BatchedPlan", "mr1l_plan", "mr1l_construct", "memory_cache", "work_limit", "batch_inblock",
           "version"]

_DT = {"c64": (_lib.C64, torch.complex64), "c128": (_lib.C128, torch.complex128)}
_W = {"paper": _lib.W_PAPER, "eval": _lib.W_EVAL}


def _stream(device: torch.device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor | None) -> C.c_void_p:
    return C.c_void_p(0 if t is None else t.data_ptr())


def version() -> str:
    return lib().mr1l_version().decode()


def memory_cache(device: int = 0, max_idle_bytes: int = -1) -> int:
    """Return the idle blocks of the library's device-memory cache on ``device`` to the driver and
    set the cap on idle bytes (< 0 keeps it, 0 disables caching); returns the bytes released."""
    out = C.c_int64(0)
    check(lib().mr1l_memory_cache(int(device), int(max_idle_bytes), C.byref(out)), "mr1l_memory_cache")
    return int(out.value)


def work_limit(max_bytes: int = 0) -> int:
    """mr1l_work_limit: bound of the Bluestein work area of plans created from now on (> 0 sets it,
    < 0 restores the default, 0 queries); returns the bound in effect."""
    out = C.c_int64(0)
    check(lib().mr1l_work_limit(int(max_bytes), C.byref(out)), "mr1l_work_limit")
    return int(out.value)


def batch_inblock(enable: int = -1) -> int:
    """mr1l_batch_inblock: whether batched plans created from now on run their small transforms in
    the persistent in-block kernel (1 on, 0 off, < 0 query); returns the setting."""
    out = C.c_int(0)
    check(lib().mr1l_batch_inblock(int(enable), C.byref(out)), "mr1l_batch_inblock")
    return int(out.value)


def fft_smooth(mode: int = -1) -> int:
    """mr1l_fft_smooth: whether plans created from now on may take Bluestein lengths 3 * 2^k
    (1 where the tuned table says so, 2 wherever the lattices fit, 0 powers of two only, < 0
    query); returns the mode."""
    out = C.c_int(0)
    check(lib().mr1l_fft_smooth(int(mode), C.byref(out)), "mr1l_fft_smooth")
    return int(out.value)


def rhs_interleave(mode: int = -1) -> int:
    """mr1l_rhs_interleave: whether plans created from now on read several right-hand sides per
    random access in the gather and the Fourier-matrix adjoint (1 by size, 2 every pass of several
    right-hand sides, 0 never, < 0 query); returns the mode."""
    out = C.c_int(0)
    check(lib().mr1l_rhs_interleave(int(mode), C.byref(out)), "mr1l_rhs_interleave")
    return int(out.value)


class Plan:
    """mr1l_plan: frequency set I (int [n, d]), lattices (M [L], z [L, d])."""

    def __init__(self, freqs, M, z, dtype: str = "c64", weights: str = "paper", n_rhs: int = 1,
                 device: int | torch.device | None = None):
        f = np.ascontiguousarray(np.asarray(freqs, dtype=np.int32))
        if f.ndim != 2:
            raise ValueError("freqs must be [n, d]")
        self.n, self.d = int(f.shape[0]), int(f.shape[1])
        Mv = np.ascontiguousarray(np.asarray(M, dtype=np.int64).reshape(-1))
        zv = np.ascontiguousarray(np.asarray(z, dtype=np.int64).reshape(len(Mv), self.d))
        self.L = int(len(Mv))
        self.M = Mv
        self.z = zv
        self.dtype_name = dtype
        self.code, self.torch_dtype = _DT[dtype]
        self.weights = weights
        self.n_rhs = int(n_rhs)
        if device is None:
            device = torch.cuda.current_device()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        handle = C.c_void_p()
        check(lib().mr1l_plan(self.d, self.n, f.ctypes.data_as(C.c_void_p), self.L,
                              Mv.ctypes.data_as(C.c_void_p), zv.ctypes.data_as(C.c_void_p), self.code,
                              _W[weights], self.n_rhs, self.device.index, C.byref(handle)), "mr1l_plan")
        self._h = handle
        self.max_nlat = self.L
        self._finish()

    def _finish(self):
        off = np.zeros(self.L + 1, np.int64)
        lens = np.zeros(max(1, self.L), np.int64)
        check(lib().mr1l_info(self._h, off.ctypes.data_as(C.c_void_p), None, lens.ctypes.data_as(C.c_void_p)),
              "mr1l_info")
        self.sample_offsets = off
        self.fft_lengths = lens[: self.L]
        self.sum_M = int(off[-1])

    # -- helpers ----------------------------------------------------------------------------------
    def _check_tensor(self, t: torch.Tensor, last: int, what: str) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError(f"{what} must be a tensor on {self.device}")
        if t.dtype != self.torch_dtype:
            raise ValueError(f"{what} must be {self.torch_dtype}")
        if t.dim() == 1:
            t = t.reshape(1, -1)
        if tuple(t.shape) != (self.n_rhs, last):
            raise ValueError(f"{what} must have shape ({self.n_rhs}, {last}), got {tuple(t.shape)}")
        return t.contiguous()

    def empty_samples(self) -> torch.Tensor:
        return torch.empty((self.n_rhs, self.sum_M), dtype=self.torch_dtype, device=self.device)

    def empty_coeffs(self) -> torch.Tensor:
        return torch.empty((self.n_rhs, self.n), dtype=self.torch_dtype, device=self.device)

    # -- transforms -------------------------------------------------------------------------------
    def forward(self, samples: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """mr1l_forward: samples [n_rhs, sum M] -> coefficients [n_rhs, n]."""
        y = self._check_tensor(samples, self.sum_M, "samples")
        c = self.empty_coeffs() if out is None else self._check_tensor(out, self.n, "out")
        check(lib().mr1l_forward(self._h, _ptr(y), _ptr(c), _stream(self.device)), "mr1l_forward")
        return c

    def adjoint(self, coeffs: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """mr1l_adjoint: coefficients [n_rhs, n] -> samples [n_rhs, sum M]."""
        c = self._check_tensor(coeffs, self.n, "coeffs")
        y = self.empty_samples() if out is None else self._check_tensor(out, self.sum_M, "out")
        check(lib().mr1l_adjoint(self._h, _ptr(c), _ptr(y), _stream(self.device)), "mr1l_adjoint")
        return y

    def lsq_residual(self, s: torch.Tensor, y: torch.Tensor, grad: torch.Tensor | None = None,
                     loss: torch.Tensor | None = None, scale: torch.Tensor | None = None) -> None:
        """mr1l_lsq_residual: loss = 1/2 sum (1/M_l) |s - y|^2 into ``loss`` (float64 scalar tensor)
        and/or grad = scale (1/M_l)(s - y) into ``grad`` (may be ``s``); ``scale`` a float64
        scalar tensor on the device (None: 1)."""
        s = self._check_tensor(s, self.sum_M, "s")
        y = self._check_tensor(y, self.sum_M, "y")
        if grad is not None:
            grad = self._check_tensor(grad, self.sum_M, "grad")
        for t, name in ((loss, "loss"), (scale, "scale")):
            if t is not None and (t.dtype != torch.float64 or t.numel() != 1 or t.device != s.device
                                  or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float64 scalar tensor on the plan's device")
        check(lib().mr1l_lsq_residual(self._h, _ptr(s), _ptr(y), _ptr(scale), _ptr(grad), _ptr(loss),
                                      _stream(self.device)), "mr1l_lsq_residual")

    def alias(self):
        """mr1l_alias: (residues int64 [L, n], unaliased uint8 [L, n], counter uint8 [n]) on device."""
        res = torch.empty((self.max_nlat, self.n), dtype=torch.int64, device=self.device)
        uniq = torch.empty((self.max_nlat, self.n), dtype=torch.uint8, device=self.device)
        cnt = torch.empty((self.n,), dtype=torch.uint8, device=self.device)
        check(lib().mr1l_alias(self._h, _ptr(res), _ptr(uniq), _ptr(cnt), _stream(self.device)), "mr1l_alias")
        return res, uniq, cnt

    def n_uncovered(self) -> int:
        u = C.c_int64(0)
        check(lib().mr1l_info(self._h, None, C.byref(u), None), "mr1l_info")
        return int(u.value)

    # -- graph capture ----------------------------------------------------------------------------
    def capture(self, direction: str, inp: torch.Tensor, out: torch.Tensor):
        """Record one forward or adjoint call (its fixed set of kernel launches) into a HIP graph
        through torch.cuda.CUDAGraph; replay() then reruns it on the same buffers."""
        fn = self.forward if direction == "forward" else self.adjoint
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):
            fn(inp, out=out)
        torch.cuda.current_stream(self.device).wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn(inp, out=out)
        return g

    # -- timing -----------------------------------------------------------------------------------
    def cache_alias(self, enable: bool = True) -> None:
        """Reuse the residues and alias bitmaps between calls (they depend only on the frequency
        set and the lattices); off by default, where every call recomputes them as Alg. 2 does."""
        check(lib().mr1l_cache_alias(self._h, int(enable)), "mr1l_cache_alias")

    def timing(self, enable: bool = True) -> None:
        check(lib().mr1l_timing_enable(self._h, int(enable)), "mr1l_timing_enable")

    def timing_read(self) -> dict:
        ms = (C.c_double * _lib.NSTAGES)()
        cnt = (C.c_int64 * _lib.NSTAGES)()
        names = (C.c_char_p * _lib.NSTAGES)()
        check(lib().mr1l_timing_read(self._h, ms, cnt, names), "mr1l_timing_read")
        return {names[i].decode(): (ms[i], int(cnt[i])) for i in range(_lib.NSTAGES) if cnt[i]}

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().mr1l_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedPlan(Plan):
    """mr1l_plan_batched: independent transforms [(freqs_b, M_b, z_b), ...] in one plan; samples
    and coefficients of the transforms are stacked one after another."""

    def __init__(self, problems, dtype: str = "c64", weights: str = "paper", n_rhs: int = 1,
                 device: int | torch.device | None = None):
        d = int(np.asarray(problems[0][0]).shape[1])
        fl = [np.asarray(p[0], np.int32).reshape(-1, d) for p in problems]
        Ml = [np.asarray(p[1], np.int64).reshape(-1) for p in problems]
        zl = [np.asarray(p[2], np.int64).reshape(len(m), d) for p, m in zip(problems, Ml)]
        self.tx_n = np.array([f.shape[0] for f in fl], np.int64)
        self.tx_L = np.array([len(m) for m in Ml], np.int32)
        f = np.ascontiguousarray(np.concatenate(fl)) if len(fl) else np.zeros((0, d), np.int32)
        Mv = np.ascontiguousarray(np.concatenate(Ml))
        zv = np.ascontiguousarray(np.concatenate(zl))
        self.n, self.d, self.L = int(f.shape[0]), d, int(len(Mv))
        self.M, self.z = Mv, zv
        self.dtype_name = dtype
        self.code, self.torch_dtype = _DT[dtype]
        self.weights = weights
        self.n_rhs = int(n_rhs)
        if device is None:
            device = torch.cuda.current_device()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        handle = C.c_void_p()
        check(lib().mr1l_plan_batched(d, len(problems), self.tx_n.ctypes.data_as(C.c_void_p),
                                      f.ctypes.data_as(C.c_void_p), self.tx_L.ctypes.data_as(C.c_void_p),
                                      Mv.ctypes.data_as(C.c_void_p), zv.ctypes.data_as(C.c_void_p), self.code,
                                      _W[weights], self.n_rhs, self.device.index, C.byref(handle)),
              "mr1l_plan_batched")
        self._h = handle
        self.max_nlat = int(self.tx_L.max()) if len(self.tx_L) else 0
        self.freq_offsets = np.concatenate([[0], np.cumsum(self.tx_n)])
        self.lat_offsets = np.concatenate([[0], np.cumsum(self.tx_L)])
        self._finish()


def mr1l_plan(*args, **kwargs) -> Plan:
    return Plan(*args, **kwargs)


def mr1l_construct(freqs, c: float = 2.0, gamma: float = 0.5, b: int = 10, seed: int = 0, t: int = 0,
                   device: int = 0, redraw: int = 0):
    """Alg. 1 with up to b calls (redraw > 0: the variant that redraws z_L while the lattice adds
    no reconstructible frequency).  Returns (M [L], z [L, d], calls, n_uncovered)."""
    f = np.ascontiguousarray(np.asarray(freqs, dtype=np.int32))
    n, d = f.shape
    cap = 256
    M = np.zeros(cap, np.int64)
    z = np.zeros((cap, d), np.int64)
    L = C.c_int(0)
    calls = C.c_int(0)
    unc = C.c_int64(0)
    check(lib().mr1l_construct(d, n, f.ctypes.data_as(C.c_void_p), c, gamma, b, redraw, seed, t, cap, C.byref(L),
                               M.ctypes.data_as(C.c_void_p), z.ctypes.data_as(C.c_void_p), C.byref(calls),
                               C.byref(unc), device), "mr1l_construct")
    return M[: L.value].copy(), z[: L.value].copy(), int(calls.value), int(unc.value)
