"""GPU parity at the workloads' full sizes, on sampled channels.

* A one-second integration of complex float32 samples (192 blocks of 256
  samples, 49 152 samples; Section 2 integrates about one second) folded
  block by block through the streaming server, and through repeated
  accumulate-mode calls (Section 4.5 accumulates sub-interval results), held
  to the single-precision bar (1e-5 normwise) against the FP64 oracle over the
  whole integration.  The errors are printed for the record.
* The 32-sub-array batch draw (stations 24..576, channels 16..1024, 768
  samples), complex int8 (bit-exact) and complex float32 (1e-5), checked on
  two random channels per sub-array.
* A fold of the streaming workload's shape (512 stations, 4096 channels,
  blocks of 256 samples), checked on sampled channels.
* The XC_CHECK=1 scan rejecting -128 in int8 input.
"""
import os
import time

import numpy as np
import pytest
import torch

import paper_1702_00844_amd as xe
from paper_1702_00844_amd import inputs
from tests.helpers import gpu_vis_numpy, oracle_vis, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
FP32_TOL = 1e-5


def _cs_err(got, ref, S):
    """Largest |dV_ij,pq| / sqrt(V_ii,pp V_jj,qq) (Cauchy-Schwarz normalised)."""
    auto = np.array([ref[:, s * (s + 1) // 2 + s] for s in range(S)])       # [S, C, 2, 2]
    pw = np.stack([auto[..., 0, 0].real, auto[..., 1, 1].real], axis=-1)    # [S, C, 2]
    worst = 0.0
    for j in range(S):
        for i in range(j + 1):
            b = j * (j + 1) // 2 + i
            scale = np.sqrt(pw[i][:, :, None] * pw[j][:, None, :])          # [C, 2, 2]
            worst = max(worst, float(np.max(np.abs(got[:, b] - ref[:, b]) / scale)))
    return worst


def test_fp32_one_second_integration_drift():
    """FP32 resident accumulators over 49 152 samples: the folded result and
    the accumulate-mode result both stay within 1e-5 of the FP64 oracle, so no
    FP64 cross-block accumulator is needed."""
    S, C, bt, bpi, k = 64, 3, 256, 192, 8
    blocks = [inputs.cn_gaussian(C, bt, S, seed=20000 + b, device=DEV) for b in range(bpi)]
    whole = torch.cat(blocks, dim=1)
    ref = oracle_vis(whole)

    # through the streaming server (staggered folds of 8 blocks)
    srv = xe.Server()
    d = xe.Server.desc(S, C, bt, bpi, blocks_per_fold=k, in_type=xe.XC_IN_CF32, acc_type=xe.XC_OUT_CF32,
                       staggered=True)
    sid = srv.open(d)
    for b in range(bpi):
        while True:
            try:
                ptr = srv.acquire(sid)
                break
            except xe.XengineError as e:
                assert e.status_name == "XC_ERR_BACKPRESSURE"
                time.sleep(0.0005)
        xe.device_tensor(ptr, (C, bt, S, 4), torch.float32).copy_(torch.view_as_real(blocks[b]).reshape(C, bt, S, 4))
        torch.cuda.synchronize()
        srv.commit(sid, time.monotonic_ns())
    srv.stats(sid)
    vptr, seq = srv.latest(sid)
    assert seq == 0
    got_srv = gpu_vis_numpy(xe.device_tensor(vptr, xe.vis_shape(C, S, xe.XC_OUT_CF32), torch.complex64))
    srv.close()

    # repeated accumulate-mode calls, one per block
    out = torch.zeros(xe.vis_shape(C, S, xe.XC_OUT_CF32), dtype=torch.complex64, device=DEV)
    for b in range(bpi):
        xe.correlate_into(blocks[b], out, accumulate=True)
    torch.cuda.synchronize()
    got_acc = gpu_vis_numpy(out)
    # one call over the whole integration, for comparison
    got_one = gpu_vis_numpy(xe.correlate(whole))

    errs = {}
    for name, got in (("server_folds", got_srv), ("accumulate_per_block", got_acc), ("single_call", got_one)):
        errs[name] = (rel_err(got, ref), _cs_err(got, ref, S))
        print(f"{name}: normwise {errs[name][0]:.3e}, worst Cauchy-Schwarz-normalised {errs[name][1]:.3e}")
    for name, (nw, cs) in errs.items():
        assert nw <= FP32_TOL, (name, nw)


def _sampled(rng, C, n=2):
    return sorted(rng.choice(C, size=min(n, C), replace=False).tolist())


@pytest.mark.parametrize("kind", ["ci8", "cf32"])
def test_batch_draw_sampled_channels(kind):
    """The 32-sub-array draw in one batch plan (graph-replayed, as the
    benchmark times it): two random channels of every sub-array against the
    oracle."""
    shapes = inputs.subarray_shapes(32, seed=4)
    rng = np.random.default_rng(44)
    xs, outs = [], []
    for k, (S, C, T) in enumerate(shapes):
        if kind == "ci8":
            xs.append(inputs.ci8_gaussian(C, T, S, seed=4000 + k, device=DEV, chunk_channels=128))
            outs.append(torch.empty(xe.vis_shape(C, S, xe.XC_OUT_CI32), dtype=torch.int32, device=DEV))
        else:
            xs.append(inputs.cn_gaussian(C, T, S, seed=4000 + k, device=DEV))
            outs.append(torch.empty(xe.vis_shape(C, S, xe.XC_OUT_CF32), dtype=torch.complex64, device=DEV))
    plan = xe.BatchPlan(xs, outs, use_graph=True)
    plan.run()
    torch.cuda.synchronize()
    plan.close()
    for k, (S, C, T) in enumerate(shapes):
        ch = _sampled(rng, C)
        ref = oracle_vis(xs[k], channels=ch)
        got = gpu_vis_numpy(outs[k], channels=ch)
        if kind == "ci8":
            assert np.array_equal(got, ref), (k, S, C, ch)
        else:
            assert rel_err(got, ref) <= FP32_TOL, (k, S, C, ch, rel_err(got, ref))
    del xs, outs
    torch.cuda.empty_cache()


def test_stream_workload_fold_sampled_channels():
    """Streaming workload shape: 512 stations, 4096 channels, complex int8
    blocks of 256 samples, staggered folds of 4 blocks, integrations of 8
    blocks (two of them, the second in the other resident buffer): sampled
    channels of both integrations bit-exact against the oracle."""
    S, C, bt, bpi, k = 512, 4096, 256, 8, 4
    rng = np.random.default_rng(55)
    ch = sorted(set(_sampled(rng, C, 3) + [0, C - 1]))
    srv = xe.Server()
    d = xe.Server.desc(S, C, bt, bpi, blocks_per_fold=k, ring_blocks=2 * k, staggered=True)
    sid = srv.open(d)
    kept = []
    for b in range(2 * bpi):
        blk = inputs.ci8_gaussian(C, bt, S, seed=5000 + b, device=DEV, chunk_channels=256)
        kept.append(blk[ch].cpu())
        while True:
            try:
                ptr = srv.acquire(sid)
                break
            except xe.XengineError as e:
                assert e.status_name == "XC_ERR_BACKPRESSURE"
                time.sleep(0.001)
        xe.device_tensor(ptr, (C, bt, S, 2, 2), torch.int8).copy_(blk)
        del blk
        torch.cuda.synchronize()
        srv.commit(sid, time.monotonic_ns())
        if (b + 1) % bpi == 0:
            n = (b + 1) // bpi - 1
            srv.stats(sid)
            vptr, _ = srv.integration(sid, n)
            v = xe.device_tensor(vptr, xe.vis_shape(C, S, xe.XC_OUT_CI32), torch.int32)
            got = gpu_vis_numpy(v, channels=ch)
            ref = oracle_vis(torch.cat(kept[b + 1 - bpi:b + 1], dim=1))
            assert np.array_equal(got, ref), n
    srv.close()
    torch.cuda.empty_cache()


def test_xc_check_rejects_minus_128(monkeypatch):
    """XC_CHECK=1 scans int8 input: -128 (outside the [-127, 127] domain that
    makes the matrix-core imaginary part exact) is rejected before the
    correlation is launched; valid input passes."""
    x = inputs.ci8_gaussian(3, 40, 12, seed=9, device=DEV)
    monkeypatch.setenv("XC_CHECK", "1")
    v = xe.correlate(x)
    torch.cuda.synchronize()
    assert np.array_equal(gpu_vis_numpy(v), oracle_vis(x))
    x[1, 17, 5, 1, 0] = -128
    out = torch.full_like(v, 7)
    with pytest.raises(xe.XengineError) as e:
        xe.correlate_into(x, out)
    assert e.value.status_name == "XC_ERR_INVALID_ARG" and "-128" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(out == 7)          # nothing was launched
    monkeypatch.delenv("XC_CHECK")
