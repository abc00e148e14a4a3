"""GPU tests of the batch plans (one workgroup per unit, hipGraph replay), the
auto-tuner and the streaming server, against the oracle."""
import ctypes
import os
import time

import numpy as np
import pytest
import torch

import paper_1702_00844_amd as xe
from paper_1702_00844_amd import _lib, inputs
from tests.helpers import gpu_vis_numpy, oracle_vis, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

SHAPES = [(24, 5, 768), (70, 3, 300), (130, 2, 128), (8, 16, 256), (1, 4, 33), (65, 1, 1000)]
# station counts that are multiples of 4: int8 and 16-bit batches run the direct-to-LDS kernels
SHAPES4 = [(24, 5, 768), (68, 3, 300), (132, 2, 128), (8, 16, 256), (4, 4, 33), (64, 1, 1000)]


def _make(kind, shapes, seed=40):
    xs = []
    for k, (S, C, T) in enumerate(shapes):
        if kind == "ci8":
            xs.append(inputs.ci8_gaussian(C, T, S, seed=seed + k, device=DEV))
        elif kind == "cf32":
            xs.append(inputs.cn_gaussian(C, T, S, seed=seed + k, device=DEV))
        else:
            dt = torch.float16 if kind == "cf16" else torch.bfloat16
            xs.append(inputs.ci8_gaussian(C, T, S, seed=seed + k, device=DEV).to(dt))
    return xs


def _check(kind, xs, outs, base=None):
    for k, (x, o) in enumerate(zip(xs, outs)):
        src = x.to(torch.int8) if kind in ("cf16", "cbf16") else x
        ref = oracle_vis(src)
        if base is not None:
            ref = ref + base[k]
        got = gpu_vis_numpy(o)
        if kind == "ci8":
            assert np.array_equal(got, ref), k
        elif kind in ("cf16", "cbf16"):
            assert np.array_equal(got, ref[..., 0] + 1j * ref[..., 1]), k
        else:
            assert rel_err(got, ref) <= 1e-5, k


@pytest.mark.parametrize("kind,config,shapes", [
    ("ci8", None, SHAPES4), ("ci8", None, SHAPES), ("cf16", None, SHAPES4), ("cf16", None, SHAPES),
    ("cbf16", None, SHAPES),
    ("cf32", {"kernel": xe.XC_KERNEL_MFMA, "block": 32}, SHAPES),
    ("cf32", {"kernel": xe.XC_KERNEL_MFMA, "block": 64, "time_split": 1}, SHAPES),
    ("cf32", {"kernel": xe.XC_KERNEL_MFMA, "block": 64, "time_split": 2}, SHAPES),
    ("cf32", {"kernel": xe.XC_KERNEL_VALU, "time_chunk": 32, "time_split": 8}, SHAPES),
    ("cf32", {"kernel": xe.XC_KERNEL_VALU, "time_chunk": 16, "time_split": 1}, SHAPES),
    ("cf32", {"kernel": xe.XC_KERNEL_MFMA, "block": 64, "time_split": 2, "product": xe.XC_PRODUCT_FOUR}, SHAPES),
    ("ci8", {"kernel": xe.XC_KERNEL_MFMA, "block": 64, "staging": xe.XC_STAGING_REGISTERS}, SHAPES),
    ("ci8", {"kernel": xe.XC_KERNEL_MFMA, "block": 32}, SHAPES4),
    ("cf16", {"kernel": xe.XC_KERNEL_MFMA, "block": 64, "staging": xe.XC_STAGING_REGISTERS}, SHAPES4),
], ids=["ci8_lds", "ci8_mixed", "cf16_lds", "cf16_mixed", "cbf16", "f32mfma32", "f32mfma64ts1", "f32mfma64ts2", "valu_ts8",
        "valu_ts1", "f32mfma64ts2_p4", "ci8_regs", "ci8_b32", "cf16_regs"])
@pytest.mark.parametrize("use_graph", [True, False], ids=["graph", "direct"])
def test_batch_matches_oracle(kind, config, shapes, use_graph):
    xs = _make(kind, shapes)
    out_dtype = torch.int32 if kind == "ci8" else torch.complex64
    ot = xe.XC_OUT_CI32 if kind == "ci8" else xe.XC_OUT_CF32
    outs = [torch.full(xe.vis_shape(s[1], s[0], ot), 7, dtype=out_dtype, device=DEV) for s in shapes]
    plan = xe.BatchPlan(xs, outs, config=config, use_graph=use_graph)
    assert plan.units == len(xe.batch_worklist(shapes, xe.resolve_config(
        (xe.in_type_of(xs[0])[0], 1, 1, 1, 2), ot, config)["block"]))
    for rep in range(3):
        for o in outs:
            o.fill_(3)                       # eager work between replays
        torch.cuda.synchronize()
        plan.run()
        torch.cuda.synchronize()
        _check(kind, xs, outs)
    plan.close()


def test_batch_mixes_the_small_array_kernel():
    """Complex float32 with the default configuration: sub-arrays of at most
    16 stations take the one-channel kernel, the others the matrix cores, in
    one plan (one launch per configuration), replayed from a graph."""
    shapes = [(8, 5, 100), (16, 3, 300), (40, 2, 64), (1, 7, 129), (70, 1, 33)]
    xs = _make("cf32", shapes, seed=70)
    outs = [torch.full(xe.vis_shape(s[1], s[0], xe.XC_OUT_CF32), 7, dtype=torch.complex64, device=DEV)
            for s in shapes]
    plan = xe.BatchPlan(xs, outs, use_graph=True)
    for rep in range(2):
        for o in outs:
            o.fill_(3)
        torch.cuda.synchronize()
        plan.run()
        torch.cuda.synchronize()
        _check("cf32", xs, outs)
    plan.close()


def test_stream_of_a_small_array():
    """A 12-station complex-float32 stream (folded by the one-channel kernel
    through the ring's time-blocked addressing) equals the oracle."""
    S, C, bt, bpi, k = 12, 3, 40, 4, 2
    srv = xe.Server()
    sid = srv.open(xe.Server.desc(S, C, bt, bpi, blocks_per_fold=k, ring_blocks=5, in_type=xe.XC_IN_CF32,
                                  acc_type=xe.XC_OUT_CF32, block_period_s=0.001, staggered=True))
    blocks = [inputs.cn_gaussian(C, bt, S, seed=300 + b, device=DEV) for b in range(2 * bpi)]
    for blk in blocks:
        ptr = _acquire(srv, sid)
        _fill_slot(ptr, blk, "cf32", C, bt, S)
        torch.cuda.synchronize()
        srv.commit(sid, time.monotonic_ns())
    for n in range(2):
        vptr = srv.wait_integration(sid, n, stream=torch.cuda.current_stream())
        got = xe.device_tensor(vptr, xe.vis_shape(C, S, xe.XC_OUT_CF32), torch.complex64).clone()
        torch.cuda.synchronize()
        ref = oracle_vis(torch.cat(blocks[n * bpi:(n + 1) * bpi], dim=1))
        assert rel_err(gpu_vis_numpy(got), ref) <= 1e-5, n
    srv.close()


def test_batch_accumulate():
    xs = _make("ci8", SHAPES, seed=90)
    base = [torch.randint(-1000, 1000, xe.vis_shape(s[1], s[0], xe.XC_OUT_CI32), dtype=torch.int32, device=DEV)
            for s in SHAPES]
    outs = [b.clone() for b in base]
    plan = xe.BatchPlan(xs, outs, accumulate=True, use_graph=True)
    plan.run()
    torch.cuda.synchronize()
    _check("ci8", xs, outs, base=[b.cpu().numpy().astype(np.int64) for b in base])


def test_batch_rejects_mixed_types():
    xs = [inputs.ci8_gaussian(2, 16, 8, seed=1, device=DEV), inputs.cn_gaussian(2, 16, 8, seed=1, device=DEV)]
    outs = [torch.empty(xe.vis_shape(2, 8, 1), dtype=torch.int32, device=DEV),
            torch.empty(xe.vis_shape(2, 8, 0), dtype=torch.complex64, device=DEV)]
    with pytest.raises(ValueError):
        xe.BatchPlan(xs, outs)


def test_autotune_and_cache(tmp_path):
    S, C, T = 48, 8, 256
    x = inputs.cn_gaussian(C, T, S, seed=77, device=DEV)
    out = torch.empty(xe.vis_shape(C, S, 0), dtype=torch.complex64, device=DEV)
    path = str(tmp_path / "tune.jsonl")
    best, ms = xe.autotune(x, out, cache_path=path)
    assert ms > 0 and best["kernel"] in (xe.XC_KERNEL_VALU, xe.XC_KERNEL_MFMA)
    assert os.path.exists(path) and xe.tune_cache_load(path) == 1
    v = xe.correlate(x)                      # AUTO now uses the tuned choice
    torch.cuda.synchronize()
    assert rel_err(gpu_vis_numpy(v), oracle_vis(x)) <= 1e-5


@pytest.mark.parametrize("via", ["argument", "environment"])
def test_batch_plan_tunes_buckets_into_cache(tmp_path, monkeypatch, via):
    """A batch plan without a configuration but with a tuning cache (the
    argument, or XC_TUNE_CACHE) tunes each missing shape bucket, appends it to
    the cache, and runs every item in its tuned configuration: results match
    the oracle."""
    path = str(tmp_path / "tune.jsonl")
    # shapes in buckets no other test tunes (a bucket tuned earlier in the
    # process is not tuned again, so nothing would be written)
    shapes = [(24, 5, 768), (70, 3, 300)] if via == "argument" else [(40, 4, 1500), (100, 2, 2100)]
    xs = _make("cf32", shapes, seed=140)
    outs = [torch.empty(xe.vis_shape(s[1], s[0], xe.XC_OUT_CF32), dtype=torch.complex64, device=DEV) for s in shapes]
    if via == "environment":
        monkeypatch.setenv("XC_TUNE_CACHE", path)
        plan = xe.BatchPlan(xs, outs, use_graph=True)
    else:
        monkeypatch.delenv("XC_TUNE_CACHE", raising=False)
        plan = xe.BatchPlan(xs, outs, use_graph=True, tune_cache=path)
    plan.run()
    torch.cuda.synchronize()
    plan.close()
    assert os.path.exists(path)
    assert xe.tune_cache_load(path) == len(shapes)
    _check("cf32", xs, outs)


def _fill_slot(ptr, blk, kind, C, bt, S):
    if kind == "ci8":
        xe.device_tensor(ptr, (C, bt, S, 2, 2), torch.int8).copy_(blk)
    elif kind != "cf32":
        # 16-bit samples copied bit for bit (there is no bfloat16 array-interface type)
        xe.device_tensor(ptr, (C, bt, S, 2, 2), torch.int16).copy_(blk.view(torch.int16))
    else:
        slot = xe.device_tensor(ptr, (C, bt, S, 2 * 2), torch.float32)
        slot.copy_(torch.view_as_real(blk).reshape(C, bt, S, 4))


def _acquire(srv, sid):
    while True:
        try:
            return srv.acquire(sid)
        except xe.XengineError as e:
            assert e.status_name == "XC_ERR_BACKPRESSURE"
            time.sleep(0.001)


# block_times 24: the int8 kernel's 64-step chunks straddle the ring slots of a
# fold; k = 3 with a ring of 7 slots makes folds wrap around the ring's end;
# staggered folds give each channel group its own fold boundaries ("spread":
# staggered with the groups' leftovers folded at their next turn, flushed at
# the end of every integration here)
@pytest.mark.parametrize("kind,bt,k,ring,staggered,events", [
    ("ci8", 32, 2, 4, False, False), ("ci8", 24, 2, 4, True, False), ("ci8", 24, 3, 7, True, True),
    ("cf32", 32, 2, 4, True, True), ("cf32", 16, 3, 7, False, False), ("cf16", 32, 2, 5, True, False),
    ("cbf16", 24, 2, 4, False, True), ("ci8", 24, 3, 7, "spread", True), ("cf32", 32, 2, 4, "spread", False)],
    ids=["ci8_all", "ci8_stag", "ci8_stag_wrap_ev", "cf32_stag_ev", "cf32_all_wrap", "cf16_stag", "cbf16_all_ev",
         "ci8_spread_wrap_ev", "cf32_spread"])
def test_stream_integrations_match_oracle(kind, bt, k, ring, staggered, events):
    """Every integration read back through xc_stream_integration (its ready
    event waited on by a consumer stream) equals the oracle over its blocks;
    with events, blocks are filled on a producer stream and committed with
    xc_stream_commit_after, and every integration is released."""
    S, C, bpi = 20, 5, 6
    n_int = 3
    srv = xe.Server()
    in_type = {"ci8": xe.XC_IN_CI8, "cf32": xe.XC_IN_CF32, "cf16": xe.XC_IN_CF16, "cbf16": xe.XC_IN_CBF16}[kind]
    acc = xe.XC_OUT_CI32 if kind == "ci8" else xe.XC_OUT_CF32
    d = xe.Server.desc(S, C, bt, bpi, blocks_per_fold=k, ring_blocks=ring, in_type=in_type, acc_type=acc,
                       block_period_s=0.001, staggered=bool(staggered), spread_ends=staggered == "spread")
    sid = srv.open(d)
    producer, consumer = torch.cuda.Stream(), torch.cuda.Stream()
    blocks = []
    for b in range(bpi * n_int):
        if kind == "cf32":
            blk = inputs.cn_gaussian(C, bt, S, seed=500 + b, device=DEV)
        else:
            # 16-bit samples hold the int8 values exactly, and every partial sum
            # (at most 144 x 2 x 127^2 < 2^24) is exact in float32
            blk = inputs.ci8_gaussian(C, bt, S, seed=500 + b, device=DEV)
            if kind != "ci8":
                blk = blk.to(torch.float16 if kind == "cf16" else torch.bfloat16)
        blocks.append(blk)
        ptr = _acquire(srv, sid)
        if events:
            producer.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(producer):
                _fill_slot(ptr, blk, kind, C, bt, S)
            srv.commit(sid, time.monotonic_ns(), producer_stream=producer)
        else:
            _fill_slot(ptr, blk, kind, C, bt, S)
            torch.cuda.synchronize()
            srv.commit(sid, time.monotonic_ns())
        if (b + 1) % bpi == 0:
            n = (b + 1) // bpi - 1
            if staggered == "spread":
                srv.flush(sid)
            shape = xe.vis_shape(C, S, acc)
            with torch.cuda.stream(consumer):
                vptr = srv.wait_integration(sid, n, stream=consumer)     # the host does not wait
                got = xe.device_tensor(vptr, shape, torch.int32 if kind == "ci8" else torch.complex64).clone()
                if events:
                    srv.release(sid, n, stream=consumer)
            consumer.synchronize()
            window = torch.cat(blocks[b + 1 - bpi:b + 1], dim=1)
            ref = oracle_vis(window.to(torch.int8) if kind in ("cf16", "cbf16") else window)
            if kind == "ci8":
                assert np.array_equal(gpu_vis_numpy(got), ref), n
            elif kind in ("cf16", "cbf16"):
                assert np.array_equal(gpu_vis_numpy(got), ref[..., 0] + 1j * ref[..., 1]), n
            else:
                assert rel_err(gpu_vis_numpy(got), ref) <= 1e-5, n
            assert srv.latest(sid)[1] == n
    with pytest.raises(xe.XengineError) as e:          # integration 0's buffer now holds integration 2
        srv.integration(sid, 0)
    assert e.value.status_name == "XC_ERR_STATE"
    st = srv.stats(sid)
    assert st["blocks"] == bpi * n_int and st["integrations"] == n_int and st["pending"] == 0
    folds_per_int = (bpi if staggered else bpi // k) if C >= k else None
    if folds_per_int is not None:
        # staggered: one fold per block plus the end-of-integration folds of the other groups
        expected = (bpi + (k - 1) if staggered else bpi // k) * n_int
        assert st["folds"] == expected
    assert 0 <= st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert 0 <= st["fold_p50_ms"] <= st["fold_p99_ms"] <= st["fold_max_ms"] <= st["max_ms"]
    assert st["deadline_ms"] == pytest.approx(1.0 * k)
    assert st["fold_deadline_ms"] == pytest.approx(1.0 if staggered else 1.0 * k)
    srv.reset_stats(sid)
    assert srv.stats(sid)["blocks"] == 0
    srv.close_stream(sid)
    srv.close()


def _commit_blocks(srv, sid, blocks, C, bt, S):
    for blk in blocks:
        ptr = _acquire(srv, sid)
        _fill_slot(ptr, blk, "ci8", C, bt, S)
        torch.cuda.synchronize()
        srv.commit(sid, time.monotonic_ns())


def _read_integration(srv, sid, n, C, S):
    vptr = srv.wait_integration(sid, n, stream=torch.cuda.current_stream())
    got = xe.device_tensor(vptr, xe.vis_shape(C, S, xe.XC_OUT_CI32), torch.int32).clone()
    torch.cuda.synchronize()
    return gpu_vis_numpy(got)


def test_stream_spread_ends_publish_after_the_groups_turns():
    """Spread ends (k = 3): an integration's leftovers are folded at the
    groups' next turns, so integration 0 is published with block bpi + 1 (the
    last group with a leftover), not before; integration 1, whose stream stops
    at its end, is published by xc_stream_flush.  Both equal the oracle, and
    the folds are one per block plus one extra piece per leftover."""
    S, C, bt, bpi, k = 20, 5, 24, 6, 3
    srv = xe.Server()
    sid = srv.open(xe.Server.desc(S, C, bt, bpi, blocks_per_fold=k, ring_blocks=7, block_period_s=0.001,
                                  staggered=True, spread_ends=True))
    blocks = [inputs.ci8_gaussian(C, bt, S, seed=900 + b, device=DEV) for b in range(2 * bpi)]
    _commit_blocks(srv, sid, blocks[:bpi + 1], C, bt, S)
    assert srv.latest(sid)[1] == -1          # groups 0 and 1 still hold blocks 4, 5 and 5
    _commit_blocks(srv, sid, blocks[bpi + 1:bpi + 2], C, bt, S)
    assert srv.latest(sid)[1] == 0
    ref0 = oracle_vis(torch.cat(blocks[:bpi], dim=1))
    assert np.array_equal(_read_integration(srv, sid, 0, C, S), ref0)
    _commit_blocks(srv, sid, blocks[bpi + 2:], C, bt, S)
    assert srv.latest(sid)[1] == 0
    srv.flush(sid)
    assert srv.latest(sid)[1] == 1
    ref1 = oracle_vis(torch.cat(blocks[bpi:], dim=1))
    assert np.array_equal(_read_integration(srv, sid, 1, C, S), ref1)
    st = srv.stats(sid)
    # 12 turns, blocks 6 and 7 fold two pieces each, the flush folds groups 0 and 1
    assert st["blocks"] == 2 * bpi and st["pending"] == 0 and st["folds"] == 16
    assert st["integrations"] == 2
    srv.close_stream(sid)
    srv.close()


@pytest.mark.parametrize("spread", [False, True], ids=["staggered", "spread"])
def test_stream_fold_order_across_streams(spread):
    """With the server's fold order on, two streams committed in turn (and a
    third opened and closed on the way) still produce exactly the oracle's
    integrations; the order can be switched off and on between blocks."""
    S, C, bt, bpi, k = 36, 6, 32, 4, 2
    srv = xe.Server()
    srv.set_fold_order(True)
    d = xe.Server.desc(S, C, bt, bpi, blocks_per_fold=k, ring_blocks=2 * k, block_period_s=0.001,
                       staggered=True, spread_ends=spread)
    sids = [srv.open(d), srv.open(d)]
    blocks = {sid: [inputs.ci8_gaussian(C, bt, S, seed=1300 + 97 * sid + b, device=DEV) for b in range(2 * bpi)]
              for sid in sids}
    for b in range(2 * bpi):
        if b == bpi // 2:
            extra = srv.open(d)
            _commit_blocks(srv, extra, [blocks[sids[0]][0]], C, bt, S)
            srv.close_stream(extra)
        if b == bpi:
            srv.set_fold_order(False)
        if b == bpi + 1:
            srv.set_fold_order(True)
        for sid in sids:
            _commit_blocks(srv, sid, [blocks[sid][b]], C, bt, S)
    for sid in sids:
        srv.flush(sid)
        for n in range(2):
            ref = oracle_vis(torch.cat(blocks[sid][n * bpi:(n + 1) * bpi], dim=1))
            assert np.array_equal(_read_integration(srv, sid, n, C, S), ref), (sid, n)
        st = srv.stats(sid)
        assert st["blocks"] == 2 * bpi and st["pending"] == 0
    srv.close()


def test_stream_late_arrivals_are_misses():
    """Miss accounting against a host clock moved by the test: blocks stamped
    one second in the past exceed the k P deadline, blocks stamped in the
    future complete before they 'arrive' (latency 0)."""
    S, C, bt, bpi, k = 16, 4, 32, 4, 2
    srv = xe.Server()
    d = xe.Server.desc(S, C, bt, bpi, blocks_per_fold=k, ring_blocks=4, block_period_s=0.001)
    sid = srv.open(d)
    now = time.monotonic_ns()
    for b in range(bpi):
        ptr = srv.acquire(sid)
        xe.device_tensor(ptr, (C, bt, S, 2, 2), torch.int8).zero_()
        torch.cuda.synchronize()
        srv.commit(sid, now - 1_000_000_000 if b < 2 else now + 60_000_000_000)
    st = srv.stats(sid)
    assert st["blocks"] == bpi
    assert st["misses"] == 2
    assert st["max_ms"] >= 1000.0
    assert st["p50_ms"] == 0.0      # nearest rank of [0, 0, ~1000, ~1000]
    srv.close()


def test_stream_backpressure_is_deterministic():
    """A held stream cannot finish its folds: once the ring's slots are all
    waiting for folds, acquire returns XC_ERR_BACKPRESSURE, and it succeeds
    again after the hold is released.  A hold that is never released ends at
    its time limit."""
    S, C, bt, bpi, k, ring = 16, 4, 32, 8, 2, 4
    srv = xe.Server()
    d = xe.Server.desc(S, C, bt, bpi, blocks_per_fold=k, ring_blocks=ring, staggered=False)
    sid = srv.open(d)
    blocks = [inputs.ci8_gaussian(C, bt, S, seed=900 + b, device=DEV) for b in range(bpi)]
    torch.cuda.synchronize()
    srv.hold(sid, 30.0)
    for b in range(ring):                 # fill the ring: two folds wait behind the hold
        ptr = srv.acquire(sid)
        xe.device_tensor(ptr, (C, bt, S, 2, 2), torch.int8).copy_(blocks[b])
        torch.cuda.current_stream().synchronize()      # not the device: the held stream must not be waited for
        srv.commit(sid, time.monotonic_ns())
    t0 = time.monotonic()
    for _ in range(3):
        with pytest.raises(xe.XengineError) as e:
            srv.acquire(sid)
        assert e.value.status_name == "XC_ERR_BACKPRESSURE"
    srv.resume(sid)
    for b in range(ring, bpi):
        ptr = _acquire(srv, sid)
        xe.device_tensor(ptr, (C, bt, S, 2, 2), torch.int8).copy_(blocks[b])
        torch.cuda.current_stream().synchronize()      # not the device: the held stream must not be waited for
        srv.commit(sid, time.monotonic_ns())
    assert time.monotonic() - t0 < 20.0  # released by resume, not by the time limit
    srv.stats(sid)
    vptr, seq = srv.latest(sid)
    assert seq == 0
    got = xe.device_tensor(vptr, xe.vis_shape(C, S, xe.XC_OUT_CI32), torch.int32)
    assert np.array_equal(gpu_vis_numpy(got), oracle_vis(torch.cat(blocks, dim=1)))
    # a hold nobody releases ends by itself
    srv.hold(sid, 0.05)
    t0 = time.monotonic()
    srv.stats(sid)
    assert time.monotonic() - t0 < 5.0
    srv.close()


def test_stream_state_errors_and_admission():
    srv = xe.Server()
    d = xe.Server.desc(8, 2, 16, 4, blocks_per_fold=2, ring_blocks=4)
    sid = srv.open(d)
    with pytest.raises(xe.XengineError) as e:
        srv.commit(sid, 0)
    assert e.value.status_name == "XC_ERR_STATE"
    srv.acquire(sid)
    with pytest.raises(xe.XengineError) as e:
        srv.acquire(sid)
    assert e.value.status_name == "XC_ERR_STATE"
    srv.commit(sid, time.monotonic_ns())
    srv.close_stream(sid)
    with pytest.raises(xe.XengineError):
        srv.acquire(sid)
    srv.close()
    # admission against a budget that fits exactly two such streams
    fp = xe.Server.footprint(d)
    srv = xe.Server(hbm_budget_bytes=2 * fp + fp // 2)
    a, b = srv.open(d), srv.open(d)
    with pytest.raises(xe.XengineError) as e:
        srv.open(d)
    assert e.value.status_name == "XC_ERR_ADMISSION"
    srv.close_stream(a)
    c = srv.open(d)                     # the freed budget admits a new stream
    srv.close_stream(b)
    srv.close_stream(c)
    srv.close()


def test_correlate_captured_in_a_graph():
    """xc_correlate launches captured in a HIP graph (as the launch-latency
    measurement does): every replay, with eager work in between, gives the
    eager result exactly (same kernel, same inputs)."""
    S, C, T = 8, 16, 256
    x = inputs.cn_gaussian(C, T, S, seed=1, device=DEV)
    ref = xe.correlate(x)
    out = torch.zeros_like(ref)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        xe.correlate_into(x, out, stream=side)          # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        for _ in range(4):
            xe.correlate_into(x, out, stream=side)
    for _ in range(3):
        out.zero_()                                      # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


@pytest.mark.parametrize("seed", range(6))
def test_stream_schedules_randomised(seed):
    """Two int8 streams of different shapes on one server, blocks committed in
    turn, each with a schedule drawn from {all channels, staggered, staggered
    with spread ends} and the server's fold order on or off: every integration,
    read as soon as it is published (spread ends: also after a flush at the
    end), equals the oracle bit for bit; the server publishes at the blocks
    and runs the folds that the host schedule (xc_stream_schedule) lists."""
    rng = np.random.default_rng(100 + seed)
    srv = xe.Server()
    srv.set_fold_order(bool(rng.integers(2)))
    streams = []
    for _ in range(2):
        S, C = int(rng.integers(3, 41)), int(rng.integers(1, 7))
        k = int(rng.integers(1, 5))
        bpi = k * int(rng.integers(1, 4))
        bt = int(rng.choice([8, 16, 24, 40]))
        mode = int(rng.integers(3))
        d = xe.Server.desc(S, C, bt, bpi, blocks_per_fold=k, ring_blocks=2 * k + int(rng.integers(0, 4)),
                           block_period_s=0.001, staggered=mode > 0, spread_ends=mode == 2)
        streams.append(dict(sid=srv.open(d), S=S, C=C, bt=bt, bpi=bpi, blocks=[], read=-1, desc=d))
    n_int = 3
    for st in streams:
        st["plan"] = xe.Server.schedule(st["desc"], n_int * st["bpi"], flush=True)
    for b in range(n_int * max(s["bpi"] for s in streams)):
        for st in streams:
            if len(st["blocks"]) == n_int * st["bpi"]:
                continue
            blk = inputs.ci8_gaussian(st["C"], st["bt"], st["S"], seed=int(rng.integers(1 << 30)), device=DEV)
            st["blocks"].append(blk)
            _commit_blocks(srv, st["sid"], [blk], st["C"], st["bt"], st["S"])
            nb = len(st["blocks"]) - 1
            expect = max([j for j, w in enumerate(st["plan"][1]) if 0 <= w <= nb], default=-1)
            assert srv.latest(st["sid"])[1] == expect, (nb, expect)
            _read_published(srv, st)
    for st in streams:
        srv.flush(st["sid"])
        _read_published(srv, st)
        assert st["read"] == n_int - 1
        stats = srv.stats(st["sid"])
        assert stats["pending"] == 0 and stats["integrations"] == n_int
        folds, pub = st["plan"]
        assert stats["folds"] == sum(1 for f in folds if f[3] > f[2])    # groups without channels launch nothing
        assert sum(1 for w in pub if w >= 0) == n_int
    srv.close()


def _read_published(srv, st):
    """Reads and checks every integration of stream st published since the last call."""
    latest = srv.latest(st["sid"])[1]
    for n in range(st["read"] + 1, latest + 1):
        window = torch.cat(st["blocks"][n * st["bpi"]:(n + 1) * st["bpi"]], dim=1)
        got = _read_integration(srv, st["sid"], n, st["C"], st["S"])
        assert np.array_equal(got, oracle_vis(window)), (st["S"], st["C"], n)
        st["read"] = n
