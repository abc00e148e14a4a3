"""Shared helpers of the GPU tests: move inputs to the oracle's types and
compare GPU visibilities with the oracle's."""
from __future__ import annotations

import numpy as np
import torch

import oracle


def oracle_input(x: torch.Tensor):
    """Sample tensor (any device) -> the oracle's numpy input (exact)."""
    x = x.detach().cpu()
    if x.dtype == torch.complex64:
        return x.numpy()
    if x.dtype == torch.int8:
        return x.numpy()
    # 16-bit floats: widen exactly, then pair (re, im) into complex
    f = x.to(torch.float64).numpy()
    return f[..., 0] + 1j * f[..., 1]


def oracle_vis(x: torch.Tensor, channels=None):
    """Oracle visibilities of x (optionally of a subset of channels):
    complex128 [C, B, 2, 2] for float inputs, int64 [C, B, 2, 2, 2] for int8."""
    if channels is not None:
        x = x[list(channels)]
    xi = oracle_input(x)
    if x.dtype == torch.int8:
        return oracle.correlate_i64(xi)
    return oracle.correlate_f64(xi)


def gpu_vis_numpy(v: torch.Tensor, channels=None):
    if channels is not None:
        v = v[list(channels)]
    v = v.detach().cpu()
    if v.dtype == torch.int32:
        return v.numpy().astype(np.int64)
    return v.numpy().astype(np.complex128)


def rel_err(got: np.ndarray, ref: np.ndarray) -> float:
    """Normwise relative error ||got - ref||_F / ||ref||_F."""
    if np.iscomplexobj(ref) or np.iscomplexobj(got):
        d = np.linalg.norm((got - ref).ravel())
        n = np.linalg.norm(ref.ravel())
    else:
        d = np.linalg.norm((got.astype(np.float64) - ref.astype(np.float64)).ravel())
        n = np.linalg.norm(ref.astype(np.float64).ravel())
    return float(d / n) if n > 0 else float(d)


def int_as_complex(v: np.ndarray) -> np.ndarray:
    return v[..., 0] + 1j * v[..., 1]


def assert_hermitian_autos(v: np.ndarray, S: int):
    """XX/YY autocorrelations real (imag exactly 0), YX = conj(XY) exactly."""
    if not np.iscomplexobj(v):
        v = int_as_complex(v)
    idx = [s * (s + 1) // 2 + s for s in range(S)]
    a = v[:, idx]
    assert np.all(a[..., 0, 0].imag == 0) and np.all(a[..., 1, 1].imag == 0)
    assert np.array_equal(a[..., 1, 0], np.conj(a[..., 0, 1]))
    assert np.all(a[..., 0, 0].real >= 0) and np.all(a[..., 1, 1].real >= 0)
