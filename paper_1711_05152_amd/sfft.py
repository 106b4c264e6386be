"""Python binding of sfft_detect (Alg. 3) and of the built-in planted black box.

Argument marshalling only: the 1-D projections, Alg. 1, the transforms, the selection and the
compaction all run in libmr1l on the device.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np

from . import _lib
from ._lib import check, lib

__all__ = ["sfft_detect", "SfftResult", "BsplineSum", "paper_f10"]


@dataclass
class SfftResult:
    freqs: np.ndarray          # int32 [m, d], lexicographically ascending
    coeffs: np.ndarray         # complex128 [m]
    status: int
    stats: dict = field(default_factory=dict)


def _stats_dict(st: _lib.SfftStats) -> dict:
    d = st.d
    return {
        "n_It": list(st.n_It[:d]), "n_J": list(st.n_J[:d]), "n_detected": list(st.n_detected[:d]),
        "L": list(st.L[:d]), "sumM": list(st.sumM[:d]), "calls": list(st.calls[:d]),
        "redraws": list(st.redraws[:d]),
        "uncovered": list(st.uncovered[:d]), "samples": st.samples, "samples_full": st.samples_full,
        "ms_sampling": st.ms_sampling, "ms_transform": st.ms_transform, "ms_construct": st.ms_construct,
        "ms_select": st.ms_select, "ms_total": st.ms_total,
    }


class BsplineSum:
    """Built-in test function of Sec. 5.3: f(x) = sum_tau w_tau prod_c N_{orders[tau, c]}(x_c), the
    periodic B-splines N_m normalised in L2(T) (order 0: factor 1).  Thin wrapper of the library's
    sfft_bspline description, sampler, Fourier coefficients and relative L2 error."""

    def __init__(self, orders, weights=None, dtype: str = "c128"):
        self.orders = np.ascontiguousarray(np.asarray(orders, np.int32))
        if self.orders.ndim != 2:
            raise ValueError("orders must be [terms, d]")
        self.terms, self.d = self.orders.shape
        self.weights = None if weights is None else np.ascontiguousarray(np.asarray(weights, np.float64))
        self.dtype = dtype
        self.desc = _lib.SfftBspline(terms=self.terms, d=self.d, orders=self.orders.ctypes.data,
                                     weights=None if self.weights is None else self.weights.ctypes.data,
                                     dtype={"c64": _lib.C64, "c128": _lib.C128}[dtype])

    def sample(self, nodes, out=None, stream=None):
        """f at device nodes (torch float64 [n, d]) -> torch complex [n] on the same device."""
        import torch
        if nodes.dtype != torch.float64 or nodes.dim() != 2 or nodes.shape[1] != self.d or not nodes.is_cuda:
            raise ValueError("nodes must be a CUDA float64 tensor [n, d]")
        nodes = nodes.contiguous()
        tdt = {"c64": torch.complex64, "c128": torch.complex128}[self.dtype]
        if out is None:
            out = torch.empty(nodes.shape[0], dtype=tdt, device=nodes.device)
        st = torch.cuda.current_stream(nodes.device).cuda_stream if stream is None else stream
        rc = lib().sfft_sample_bspline(C.addressof(self.desc), self.d, nodes.shape[0], nodes.data_ptr(),
                                       out.data_ptr(), st)
        if rc != 0:
            raise _lib.Mr1lError(1, "sfft_sample_bspline",
                                 lib().mr1l_last_error().decode(errors="replace"))
        return out

    def coeffs(self, freqs) -> np.ndarray:
        """Fourier coefficients f^_k (real) for the rows of freqs [n, d]."""
        f = np.ascontiguousarray(np.asarray(freqs, np.int32).reshape(-1, self.d))
        out = np.zeros((max(1, f.shape[0]), 2), np.float64)
        check(lib().sfft_bspline_coeffs(C.byref(self.desc), f.shape[0], f.ctypes.data_as(C.c_void_p),
                                        out.ctypes.data_as(C.c_void_p)), "sfft_bspline_coeffs")
        return out[:f.shape[0], 0].copy()

    def rel_l2_error(self, freqs, coeffs) -> tuple[float, float]:
        """(||f - p|| / ||f||, ||f||^2) for p = sum_k coeffs_k e^{2 pi i k.x} on the rows of freqs."""
        f = np.ascontiguousarray(np.asarray(freqs, np.int32).reshape(-1, self.d))
        c = np.asarray(coeffs, np.complex128).reshape(-1)
        cc = np.ascontiguousarray(np.stack([c.real, c.imag], axis=-1)) if len(c) else np.zeros((1, 2))
        err, nf2 = C.c_double(0.0), C.c_double(0.0)
        check(lib().sfft_bspline_l2_error(C.byref(self.desc), f.shape[0], f.ctypes.data_as(C.c_void_p),
                                          cc.ctypes.data_as(C.c_void_p), C.byref(err), C.byref(nf2)),
              "sfft_bspline_l2_error")
        return err.value, nf2.value


def paper_f10(dtype: str = "c128") -> BsplineSum:
    """The 10-variate test function of Sec. 5.3: order 2 on components 1, 3, 8, order 4 on 2, 5, 6,
    10 and order 6 on 4, 7, 9 (1-based), one product each."""
    o = np.zeros((3, 10), np.int32)
    o[0, [0, 2, 7]] = 2
    o[1, [1, 4, 5, 9]] = 4
    o[2, [3, 6, 8]] = 6
    return BsplineSum(o, dtype=dtype)


class _CudaArray:
    """__cuda_array_interface__ view of a device buffer (for caller-supplied samplers)."""

    def __init__(self, ptr: int, shape, typestr: str):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (ptr, False),
                                         "version": 3, "strides": None, "stream": None}


def sfft_detect(lo, hi, *, planted=None, sampler=None, bspline: BsplineSum | None = None, delta: float, s: int,
                s_local: int = 0, r: int = 1, b: int = 10, seed: int = 0, dtype: str = "c64",
                zero_anchors: bool = False, cap: int | None = None, device: int = 0, c: float = 2.0,
                gamma: float = 0.5, plain: bool = False, redraw: int = 0, order=None,
                delta_1d: float = 0.0) -> SfftResult:
    """Alg. 3 on the box [lo, hi].

    planted: (freqs int [s, d], coeffs complex [s], sigma, noise_seed) -- built-in black box;
    plain:   one transform call per repetition instead of repetitions as right-hand sides;
    redraw:  construction variant of step 2b (> 0: redraw z_L at most this often while the lattice
             adds no reconstructible frequency); order: component order (a permutation of 0..d-1);
    sampler: callable(nodes: torch.Tensor float64 [n, d] on the device) -> torch.Tensor complex [n]
             (used when planted is None);
    bspline: the built-in B-spline test function (its library sampler runs on the device; its dtype
             must equal ``dtype``);
    delta_1d: threshold of the 1-D detections (0: delta)."""
    lo = np.ascontiguousarray(np.asarray(lo, np.int32))
    hi = np.ascontiguousarray(np.asarray(hi, np.int32))
    d = int(lo.shape[0])
    cap = int(s if cap is None else cap)
    prm = _lib.SfftParams(delta=float(delta), s=int(s), s_local=int(s_local), r=int(r), b=int(b),
                          seed=int(seed) & ((1 << 64) - 1), dtype={"c64": _lib.C64, "c128": _lib.C128}[dtype],
                          c=float(c), gamma=float(gamma), zero_anchors=int(bool(zero_anchors)),
                          plain=int(bool(plain)), redraw=int(redraw), delta_1d=float(delta_1d))
    keep = []
    if order is not None:
        ordv = np.ascontiguousarray(np.asarray(order, np.int32).reshape(d))
        keep.append(ordv)
        prm.order = ordv.ctypes.data
    pl_ptr = None
    user = None
    if bspline is not None:
        if planted is not None or sampler is not None:
            raise ValueError("give one black box: planted, sampler or bspline")
        if bspline.dtype != dtype:
            raise ValueError("bspline.dtype must equal dtype")
        cb = C.cast(lib().sfft_sample_bspline, _lib.SAMPLER_FN)
        user = C.addressof(bspline.desc)
        keep.append(bspline)
    elif planted is not None:
        pf, pc, sigma, nseed = planted
        pf = np.ascontiguousarray(np.asarray(pf, np.int32).reshape(-1, d))
        pcc = np.ascontiguousarray(np.stack([np.real(pc), np.imag(pc)], axis=-1).astype(np.float64))
        keep += [pf, pcc]
        pl = _lib.SfftPlanted(s=int(pf.shape[0]), freqs=pf.ctypes.data, coeffs=pcc.ctypes.data, sigma=float(sigma),
                              noise_seed=int(nseed) & ((1 << 64) - 1))
        pl_ptr = C.pointer(pl)
        cb = _lib.SAMPLER_FN()
    else:
        if sampler is None:
            raise ValueError("need planted or sampler")
        import torch
        tdt = {"c64": torch.complex64, "c128": torch.complex128}[dtype]

        def _cb(user, dd, n, nodes_ptr, values_ptr, stream):
            try:
                dev = torch.device("cuda", device)
                # the library wrote the nodes on ``stream``: the caller's torch work is ordered
                # after that by running on the same stream, whatever torch's current stream is
                lib_stream = (torch.cuda.ExternalStream(stream, device=dev) if stream
                              else torch.cuda.default_stream(dev))
                with torch.cuda.stream(lib_stream):
                    x = torch.as_tensor(_CudaArray(nodes_ptr, (n, dd), "<f8"), device=dev)
                    out = torch.as_tensor(_CudaArray(values_ptr, (n, 2), "<f8" if dtype == "c128" else "<f4"),
                                          device=dev)
                    v = sampler(x).to(tdt)
                    out.copy_(torch.view_as_real(v))
                torch.cuda.synchronize(dev)
                return 0
            except Exception:  # reported as MR1L_ERR_CALLBACK
                return 1
        cb = _lib.SAMPLER_FN(_cb)
        keep.append(cb)
    f_out = np.zeros((max(1, cap), d), np.int32)
    c_out = np.zeros((max(1, cap), 2), np.float64)
    n_out = C.c_int64(0)
    st = _lib.SfftStats()
    status = lib().sfft_detect(d, lo.ctypes.data_as(C.c_void_p), hi.ctypes.data_as(C.c_void_p), cb, user, pl_ptr,
                               C.byref(prm), cap, C.byref(n_out), f_out.ctypes.data_as(C.c_void_p),
                               c_out.ctypes.data_as(C.c_void_p), C.byref(st), device)
    check(status, "sfft_detect")
    m = int(n_out.value)
    return SfftResult(f_out[:m].copy(), c_out[:m, 0] + 1j * c_out[:m, 1], status, _stats_dict(st))
