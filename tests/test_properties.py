"""Property tests over random shapes (hypothesis, derandomised so that every
run draws the same examples).

* CPU: the oracle against numpy on random shapes (complex: X X^H per channel
  in float64; int8: the exact int64 product of the real-stacked samples).
* GPU: every kernel family on random shapes, S in 1..40, C in 1..5,
  T in 1..300, each input type: complex int8 bit-exact, complex float32 within
  1e-5 normwise, and float16 / bfloat16 on integer-valued samples (exact in
  both formats and in FP32 accumulation at these sizes) bit-exact.
"""
import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle

SETTINGS = dict(deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])


def _bl(i, j):
    return j * (j + 1) // 2 + i


def _numpy_vis(x):
    """x [C, T, S, 2] complex -> [C, B, 2, 2] by the Hermitian product."""
    C, T, S, P = x.shape
    m = x.transpose(0, 2, 3, 1).reshape(C, S * P, T)             # rows (station, pol), columns time
    g = m @ np.conj(m.transpose(0, 2, 1))                          # [C, SP, SP]
    out = np.zeros((C, S * (S + 1) // 2, 2, 2), dtype=np.complex128)
    for j in range(S):
        for i in range(j + 1):
            out[:, _bl(i, j)] = g[:, i * P:(i + 1) * P, j * P:(j + 1) * P]
    return out


@settings(max_examples=60, **SETTINGS)
@given(S=st.integers(1, 12), C=st.integers(1, 3), T=st.integers(1, 40), seed=st.integers(0, 2 ** 31 - 1))
def test_oracle_f64_matches_numpy(S, C, T, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((C, T, S, 2)) + 1j * rng.standard_normal((C, T, S, 2))
    got = oracle.correlate_f64(x.astype(np.complex64))
    ref = _numpy_vis(x.astype(np.complex64).astype(np.complex128))
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * max(1.0, np.abs(ref).max()))


@settings(max_examples=60, **SETTINGS)
@given(S=st.integers(1, 12), C=st.integers(1, 3), T=st.integers(1, 40), seed=st.integers(0, 2 ** 31 - 1))
def test_oracle_i64_matches_numpy(S, C, T, seed):
    rng = np.random.default_rng(seed)
    x = rng.integers(-127, 128, size=(C, T, S, 2, 2), dtype=np.int64).astype(np.int8)
    got = oracle.correlate_i64(x)
    xc = x[..., 0].astype(np.int64) + 1j * x[..., 1].astype(np.int64)
    ref = _numpy_vis(xc.astype(np.complex128))
    assert np.array_equal(got[..., 0], np.rint(ref.real).astype(np.int64))
    assert np.array_equal(got[..., 1], np.rint(ref.imag).astype(np.int64))


# ---------------------------------------------------------------- GPU kernels
def _gpu_cases():
    import paper_1702_00844_amd as xe
    return {
        "cf32": [None, dict(kernel=xe.XC_KERNEL_VALU), dict(kernel=xe.XC_KERNEL_MFMA, block=32),
                 dict(kernel=xe.XC_KERNEL_MFMA, block=64, time_split=1)],
        "ci8": [None, dict(kernel=xe.XC_KERNEL_MFMA, block=64, staging=xe.XC_STAGING_REGISTERS),
                dict(kernel=xe.XC_KERNEL_MFMA, block=32)],
        "cf16": [None, dict(kernel=xe.XC_KERNEL_MFMA, block=32)],
        "cbf16": [None, dict(kernel=xe.XC_KERNEL_MFMA, block=32)],
    }


@pytest.mark.gpu
@settings(max_examples=120, **SETTINGS)
@given(S=st.integers(1, 40), C=st.integers(1, 5), T=st.integers(1, 300),
       kind=st.sampled_from(["cf32", "ci8", "cf16", "cbf16"]), which=st.integers(0, 3),
       seed=st.integers(0, 2 ** 31 - 1))
def test_gpu_kernels_on_random_shapes(S, C, T, kind, which, seed):
    import paper_1702_00844_amd as xe
    from paper_1702_00844_amd import inputs
    from tests.helpers import assert_hermitian_autos, gpu_vis_numpy, oracle_vis, rel_err
    cfgs = _gpu_cases()[kind]
    cfg = cfgs[which % len(cfgs)]
    dev = "cuda:0"
    if kind == "cf32":
        x = inputs.cn_gaussian(C, T, S, seed=seed % 100000, device=dev)
    else:
        xi = inputs.ci8_gaussian(C, T, S, seed=seed % 100000, device=dev)
        x = xi if kind == "ci8" else xi.to(torch.float16 if kind == "cf16" else torch.bfloat16)
    v = xe.correlate(x, config=cfg)
    torch.cuda.synchronize()
    got = gpu_vis_numpy(v)
    if kind == "cf32":
        ref = oracle_vis(x)
        assert rel_err(got, ref) <= 1e-5, (S, C, T, cfg)
    elif kind == "ci8":
        assert np.array_equal(got, oracle_vis(x)), (S, C, T, cfg)
    else:
        ref = oracle_vis(xi)                                        # integer values: exact in 16 bits
        assert np.array_equal(got, ref[..., 0] + 1j * ref[..., 1]), (S, C, T, cfg)
    assert_hermitian_autos(got, S)
