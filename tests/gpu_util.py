"""Shared helpers for the GPU parity tests (tolerances follow the precision of each path)."""
import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU (run with -m 'not gpu' here)")
    return torch


# FP64 plain path: max abs error 1e-11 on coefficients of unit scale.
# FP32 paths: normwise relative 1e-4 and max abs 1e-4 * max|ref| (entrywise relative error is
# ill-posed at near-zero entries).
def assert_close(got: np.ndarray, ref: np.ndarray, dtype: str, what: str = ""):
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    if ref.size == 0:
        return
    err = np.abs(got - ref)
    if dtype == "c128":
        scale = max(1.0, float(np.abs(ref).max()))
        assert err.max() <= 1e-11 * scale, f"{what}: max abs err {err.max():.3e} (scale {scale:.3e})"
    else:
        nref = np.linalg.norm(ref)
        if nref == 0:
            assert err.max() <= 1e-6, f"{what}: max abs err {err.max():.3e} on zero reference"
            return
        rel = np.linalg.norm(got - ref) / nref
        assert rel <= 1e-4, f"{what}: normwise rel err {rel:.3e}"
        assert err.max() <= 1e-4 * np.abs(ref).max(), f"{what}: max abs err {err.max():.3e}"
