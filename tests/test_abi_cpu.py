"""The C ABI on the CPU: every declared symbol is exported, host-only helpers
match the paper's printed values, and invalid arguments are rejected before
anything touches a device.  No GPU is needed."""
import ctypes
import math
import os
import re
import subprocess

import pytest

from paper_1702_00844_amd import _lib
import paper_1702_00844_amd as xe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xengine.h")
GOLDEN = os.path.join(ROOT, "tests", "golden")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xc_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 30
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIBRARY], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (xc_[a-z_0-9]+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, f"declared but not exported: {missing}"
    # and the binding knows every one of them
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)
    for n in names:
        getattr(lib, n)


def test_index_helpers():
    assert xe.n_baselines(64) == 2080 and xe.n_baselines(256) == 32896 and xe.n_baselines(1) == 1
    order = [(i, j) for j in range(12) for i in range(j + 1)]
    assert [xe.baseline_index(i, j) for i, j in order] == list(range(len(order)))
    assert xe.baseline_index(3, 2) == -1
    lib = _lib.load()
    assert lib.xc_vis_elems(64, 2, 256) == 256 * 2080 * 4
    assert lib.xc_sample_bytes(_lib.XC_IN_CI8, 256, 2, 1024, 1024) == 1 << 30
    assert lib.xc_sample_bytes(_lib.XC_IN_CF32, 64, 2, 256, 768) == 201326592
    assert lib.xc_vis_bytes(_lib.XC_OUT_CF32, 64, 2, 256) == 17039360


def test_table1_tile_costs():
    """Table 1: the tile cost model reproduces every printed row."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_tile_sizes.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 8
    for tile, fl, by, ai, regs in rows:
        w, h = map(int, tile.split("x"))
        f, b, r = xe.tile_cost(w, h)
        assert (f, b, r) == (int(fl), int(by), int(regs)), tile
        assert round(f / b, 2) == float(ai), tile
    # a 2x2 tile does the work of a 1x4 tile with fewer loads (Section 6)
    assert xe.tile_cost(2, 2)[0] == xe.tile_cost(1, 4)[0] and xe.tile_cost(2, 2)[1] < xe.tile_cost(1, 4)[1]
    with pytest.raises(xe.XengineError):
        xe.tile_cost(0, 3)


def test_perf_max_examples():
    rows = [l.split(None, 6) for l in open(os.path.join(GOLDEN, "perf_max.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 5
    for kind, peak, ai, bw, expect, tol, _ in rows:
        got = xe.perf_max(float(peak), float(ai), float(bw))
        assert abs(got - float(expect)) <= float(tol) + 0.01 * float(expect) * 0, (kind, peak, ai, bw, got)
    assert xe.ai_global(64) == 65.0
    assert xe.flops(64, 256, 768) == 32 * 256 * 768 * 2080


VP = ctypes.c_void_p


def call_correlate(**kw):
    args = dict(samples=VP(16), in_type=0, S=8, P=2, C=4, T=16, vis=VP(32), out_type=0, acc=0)
    args.update(kw)
    lib = _lib.load()
    return lib.xc_correlate(args["samples"], args["in_type"], args["S"], args["P"], args["C"], args["T"],
                            args["vis"], args["out_type"], args["acc"], None)


@pytest.mark.parametrize("kw,status", [
    (dict(P=1), 2), (dict(P=3), 2),
    (dict(S=0), 1), (dict(C=0), 1), (dict(T=0), 1), (dict(S=-4), 1),
    (dict(in_type=7), 1), (dict(out_type=5), 1),
    (dict(out_type=1), 1),                         # CI32 output needs int8 input
    (dict(in_type=1, out_type=1, T=66573), 4),     # int32 overflow risk
    (dict(samples=VP(0)), 1), (dict(vis=VP(0)), 1),
    (dict(samples=VP(8)), 1), (dict(vis=VP(4)), 1),  # not 16-byte aligned
    (dict(acc=2), 1),
])
def test_invalid_arguments_rejected_before_launch(kw, status):
    assert call_correlate(**kw) == status
    assert _lib.load().xc_last_error()


def test_int32_bound_is_exact():
    lib = _lib.load()
    res = _lib.XcConfig()
    assert lib.xc_resolve_config(None, 1, 1, 16, 2, 4, 66572, ctypes.byref(res)) == 0
    assert lib.xc_resolve_config(None, 1, 1, 16, 2, 4, 66573, ctypes.byref(res)) == 4
    # 2 * 127^2 * 66572 fits in int32; one more sample does not
    assert 2 * 127 * 127 * 66572 <= 2 ** 31 - 1 < 2 * 127 * 127 * 66573


def test_config_resolution():
    R, L = _lib.XC_STAGING_REGISTERS, _lib.XC_STAGING_LDS
    F4, F3 = _lib.XC_PRODUCT_FOUR, _lib.XC_PRODUCT_THREE
    shp = (_lib.XC_IN_CF32, 256, 768, 64, 2)
    r = xe.resolve_config(shp, config={"kernel": _lib.XC_KERNEL_VALU})
    assert r == {"kernel": 1, "block": 32, "time_chunk": 32, "time_split": 4, "staging": R, "product": F4,
                 "tile_w": 4, "tile_h": 2}
    r = xe.resolve_config(shp, config={"kernel": _lib.XC_KERNEL_MFMA})
    assert r == {"kernel": 2, "block": 64, "time_chunk": 32, "time_split": 2, "staging": L, "product": F3, "tile_w": 0, "tile_h": 0}
    r = xe.resolve_config((_lib.XC_IN_CF32, 1024, 1024, 256, 2), config={"kernel": _lib.XC_KERNEL_MFMA})
    assert r == {"kernel": 2, "block": 64, "time_chunk": 16, "time_split": 1, "staging": L, "product": F3, "tile_w": 0, "tile_h": 0}
    r = xe.resolve_config(shp, config={"kernel": _lib.XC_KERNEL_MFMA, "block": 32})
    assert r == {"kernel": 2, "block": 32, "time_chunk": 16, "time_split": 1, "staging": R, "product": F4, "tile_w": 0, "tile_h": 0}
    with pytest.raises(xe.XengineError):     # FP32 on 64-station blocks copies straight into LDS only
        xe.resolve_config(shp, config={"kernel": _lib.XC_KERNEL_MFMA, "staging": R})
    with pytest.raises(xe.XengineError):     # VALU stages through registers only
        xe.resolve_config(shp, config={"kernel": _lib.XC_KERNEL_VALU, "staging": L})
    with pytest.raises(xe.XengineError):
        xe.resolve_config(shp, config={"kernel": _lib.XC_KERNEL_MFMA, "staging": 3})
    with pytest.raises(xe.XengineError):
        xe.resolve_config((_lib.XC_IN_CI8, 4, 16, 8, 2), _lib.XC_OUT_CI32, config={"kernel": 2, "time_split": 2})
    # int8 and 16-bit on 64-station blocks: straight into LDS for every station
    # count (16- or 4-byte granules), through registers on request
    r = xe.resolve_config((_lib.XC_IN_CI8, 1024, 1024, 256, 2), _lib.XC_OUT_CI32)
    assert r == {"kernel": 2, "block": 64, "time_chunk": 64, "time_split": 1, "staging": L, "product": F4, "tile_w": 0, "tile_h": 0}
    r = xe.resolve_config((_lib.XC_IN_CI8, 8, 64, 70, 2), _lib.XC_OUT_CI32)
    assert r == {"kernel": 2, "block": 64, "time_chunk": 64, "time_split": 1, "staging": L, "product": F4, "tile_w": 0, "tile_h": 0}
    r = xe.resolve_config((_lib.XC_IN_CI8, 8, 64, 68, 2), _lib.XC_OUT_CI32, config={"kernel": 2, "staging": R})
    assert r == {"kernel": 2, "block": 64, "time_chunk": 64, "time_split": 1, "staging": R, "product": F4, "tile_w": 0, "tile_h": 0}
    with pytest.raises(xe.XengineError):
        xe.resolve_config((_lib.XC_IN_CI8, 8, 64, 68, 2), config={"kernel": 2, "block": 32, "staging": L})
    with pytest.raises(xe.XengineError):
        xe.resolve_config((_lib.XC_IN_CI8, 8, 64, 68, 2), config={"kernel": 2, "time_chunk": 32})
    r = xe.resolve_config((_lib.XC_IN_CF16, 1024, 1024, 256, 2))
    assert r == {"kernel": 2, "block": 64, "time_chunk": 32, "time_split": 1, "staging": L, "product": F4, "tile_w": 0, "tile_h": 0}
    r = xe.resolve_config((_lib.XC_IN_CBF16, 8, 64, 33, 2))
    assert r == {"kernel": 2, "block": 64, "time_chunk": 32, "time_split": 1, "staging": L, "product": F4, "tile_w": 0, "tile_h": 0}
    r = xe.resolve_config((_lib.XC_IN_CBF16, 8, 64, 33, 2), config={"kernel": 2, "staging": R})
    assert r == {"kernel": 2, "block": 64, "time_chunk": 32, "time_split": 1, "staging": R, "product": F4, "tile_w": 0, "tile_h": 0}
    with pytest.raises(xe.XengineError):
        xe.resolve_config((_lib.XC_IN_CI8, 4, 16, 8, 2), config={"kernel": _lib.XC_KERNEL_VALU})
    with pytest.raises(xe.XengineError):
        xe.resolve_config(shp, config={"kernel": _lib.XC_KERNEL_VALU, "time_split": 3})
    # the three-product form: complex-float32 on 64-station matrix-core blocks only
    r = xe.resolve_config(shp, config={"kernel": _lib.XC_KERNEL_MFMA, "product": F4, "tile_w": 0, "tile_h": 0})
    assert r == {"kernel": 2, "block": 64, "time_chunk": 32, "time_split": 2, "staging": L, "product": F4, "tile_w": 0, "tile_h": 0}
    r = xe.resolve_config(shp, config={"kernel": _lib.XC_KERNEL_MFMA, "time_split": 1, "product": F3, "tile_w": 0, "tile_h": 0})
    assert r == {"kernel": 2, "block": 64, "time_chunk": 16, "time_split": 1, "staging": L, "product": F3, "tile_w": 0, "tile_h": 0}
    for bad in ({"kernel": _lib.XC_KERNEL_VALU, "product": F3, "tile_w": 0, "tile_h": 0}, {"kernel": 2, "block": 32, "product": F3, "tile_w": 0, "tile_h": 0},
                {"kernel": 2, "product": 3}, {"kernel": 2, "product": -1}):
        with pytest.raises(xe.XengineError):
            xe.resolve_config(shp, config=bad)
    with pytest.raises(xe.XengineError):
        xe.resolve_config((_lib.XC_IN_CI8, 1024, 1024, 256, 2), _lib.XC_OUT_CI32, config={"product": F3, "tile_w": 0, "tile_h": 0})
    with pytest.raises(xe.XengineError):
        xe.resolve_config((_lib.XC_IN_CF16, 1024, 1024, 256, 2), config={"product": F3, "tile_w": 0, "tile_h": 0})


def test_status_strings():
    lib = _lib.load()
    for code, name in _lib.STATUS_NAMES.items():
        assert lib.xc_status_string(code).decode() == name
    assert b"gfx950" in lib.xc_version()


def test_quantile_nearest_rank():
    vals = [5.0, 1.0, 3.0, 2.0, 4.0]
    assert xe.quantile(vals, 0.5) == 3.0
    assert xe.quantile(vals, 0.99) == 5.0
    assert xe.quantile(vals, 0.0) == 1.0
    assert xe.quantile(list(range(1, 101)), 0.99) == 99
    assert math.isnan(_lib.load().xc_quantile(None, 0, 0.5))


def test_batch_worklist_covers_every_unit_once():
    shapes = [(24, 3, 768), (130, 2, 1024), (64, 5, 512), (1, 2, 10), (70, 9, 300)]
    for block in (32, 64):
        units, bounds = xe.batch_worklist(shapes, block, with_bounds=True)
        expect = set()
        for it, (S, C, T) in enumerate(shapes):
            nb = -(-S // block)
            for c in range(C):
                for bj in range(nb):
                    for bi in range(bj + 1):
                        expect.add((it, c, bi, bj))
        assert len(units) == len(expect) and set(units) == expect
        assert bounds[0] == 0 and bounds[-1] == len(units) and bounds == sorted(bounds)
        work = []
        for x in range(8):
            rng = units[bounds[x]:bounds[x + 1]]
            # longest integrations first within an XCD's range
            Ts = [shapes[u[0]][2] for u in rng]
            assert Ts == sorted(Ts, reverse=True)
            work.append(sum(shapes[u[0]][2] for u in rng))
        # every channel's block pairs are contiguous, on one XCD
        for it, (S, C, T) in enumerate(shapes):
            for c in range(C):
                pos = [k for k, u in enumerate(units) if u[0] == it and u[1] == c]
                assert pos == list(range(pos[0], pos[0] + len(pos)))
                assert sum(bounds[x] <= pos[0] < bounds[x + 1] for x in range(8)) == 1
                assert bounds[[x for x in range(8) if bounds[x] <= pos[0] < bounds[x + 1]][0] + 1] > pos[-1]
        # work dealt greedily: no XCD exceeds another by more than one channel's units
        biggest = max(T * (-(-S // block)) * (-(-S // block) + 1) // 2 for S, C, T in shapes)
        assert max(work) - min(work) <= biggest

def test_stream_footprint_and_validation():
    lib = _lib.load()
    d = xe.Server.desc(512, 4096, 256, 192, blocks_per_fold=5, ring_blocks=10)
    B = 512 * 513 // 2
    acc = 4096 * B * 4 * 8
    block = 4096 * 256 * 512 * 2 * 2
    assert xe.Server.footprint(d) == 2 * acc + 10 * block
    # budget-limited admission, checked with a server whose budget is given
    h = ctypes.c_void_p()
    assert lib.xc_server_create(1000, ctypes.byref(h)) == 0
    sid = ctypes.c_int32()
    small = xe.Server.desc(4, 2, 16, 4, blocks_per_fold=2, ring_blocks=4)
    assert xe.Server.footprint(small) > 1000
    assert lib.xc_stream_open(h, ctypes.byref(small), ctypes.byref(sid)) == 5      # XC_ERR_ADMISSION
    bad = xe.Server.desc(4, 2, 16, 5, blocks_per_fold=2, ring_blocks=4)          # 5 % 2 != 0
    assert lib.xc_stream_open(h, ctypes.byref(bad), ctypes.byref(sid)) == 1
    over = xe.Server.desc(4, 2, 256, 261, blocks_per_fold=1, ring_blocks=2)      # 66816 samples > int32 bound
    assert lib.xc_stream_open(h, ctypes.byref(over), ctypes.byref(sid)) == 4
    lib.xc_server_destroy(h)


def test_ingest_and_transpose_validation():
    """Argument errors of the host-ingest plan and the layout transpose come
    back before any device memory is touched."""
    lib = _lib.load()
    h = ctypes.c_void_p()
    TM, SM = _lib.XC_LAYOUT_TIME_MAJOR, _lib.XC_LAYOUT_STATION_MAJOR
    ok = dict(in_type=_lib.XC_IN_CF32, S=8, P=2, C=4, T=16, layout=TM, group=0)
    for bad, status in [(dict(layout=2), 1), (dict(layout=-1), 1), (dict(in_type=4), 1), (dict(P=1), 2),
                        (dict(S=0), 1), (dict(C=0), 1), (dict(T=0), 1), (dict(group=-1), 1)]:
        a = {**ok, **bad}
        assert lib.xc_ingest_create(a["in_type"], a["S"], a["P"], a["C"], a["T"], a["layout"], a["group"],
                                    ctypes.byref(h)) == status, bad
        assert not h.value
    assert lib.xc_ingest_create(0, 8, 2, 4, 16, SM, 0, None) == 1
    assert lib.xc_ingest_run(None, None, VP(16), VP(16), 0, 0, 1, None) == 1
    assert lib.xc_ingest_info(None, None, None) == 1
    lib.xc_ingest_destroy(None)
    # transpose: null or equal pointers, misalignment, bad type or shape
    for args, status in [((None, VP(64), 0, 8, 2, 1, 4), 1), ((VP(64), None, 0, 8, 2, 1, 4), 1),
                         ((VP(64), VP(64), 0, 8, 2, 1, 4), 1), ((VP(72), VP(64), 0, 8, 2, 1, 4), 1),
                         ((VP(66), VP(64), 1, 8, 2, 1, 4), 1), ((VP(64), VP(128), 5, 8, 2, 1, 4), 1),
                         ((VP(64), VP(128), 0, 8, 3, 1, 4), 2), ((VP(64), VP(128), 0, 8, 2, 1, 0), 1)]:
        assert lib.xc_transpose_to_time_major(*args, None) == status, args


def test_pfb_validation():
    """Filter-bank plans reject bad shapes before touching the device."""
    lib = _lib.load()
    h = ctypes.c_void_p()
    ok = dict(S=4, P=2, N=256, M=4, n_in=4 * 256)
    for bad, status in [(dict(N=128), 2), (dict(N=1024), 2), (dict(P=1), 2), (dict(M=0), 1), (dict(M=17), 1),
                        (dict(S=0), 1), (dict(S=16385), 1), (dict(n_in=4 * 256 - 1), 1), (dict(n_in=1 << 31), 1)]:
        a = {**ok, **bad}
        assert lib.xc_pfb_create(a["S"], a["P"], a["N"], a["M"], a["n_in"], ctypes.byref(h)) == status, bad
        assert not h.value
    assert lib.xc_pfb_create(4, 2, 256, 4, 1024, None) == 1
    assert lib.xc_pfb_run(None, VP(64), VP(64), None, VP(128), None) == 1
    assert lib.xc_pfb_info(None, None, None) == 1
    lib.xc_pfb_destroy(None)


def test_split_workspace_and_validation():
    """Pieces of ceil(T / n_split) steps, none empty; errors before any launch."""
    lib = _lib.load()
    elems = 16 * (8 * 9 // 2) * 4
    for T, n, pieces in [(10, 4, 4), (10, 6, 5), (10, 1, 1), (10, 50, 10), (1, 8, 1), (256, 16, 16), (100, 7, 7)]:
        assert lib.xc_correlate_split_bytes(8, 2, 16, T, n) == pieces * elems * 8, (T, n)
    assert lib.xc_correlate_split_bytes(8, 2, 16, 10, 0) == -1
    assert lib.xc_correlate_split_bytes(8, 3, 16, 10, 2) == -1
    # n_split < 1, null work, too small a workspace, misaligned work: rejected before anything is enqueued
    args = (None, VP(1 << 20), 0, 8, 2, 16, 10, VP(2 << 20))
    assert lib.xc_correlate_split(*args, 0, 0, 0, VP(4 << 20), 1 << 20, None) == 1
    assert lib.xc_correlate_split(*args, 0, 0, 4, None, 1 << 20, None) == 1
    assert lib.xc_correlate_split(*args, 0, 0, 4, VP(4 << 20), 16, None) == 1
    assert lib.xc_correlate_split(*args, 0, 0, 4, VP((4 << 20) + 8), 1 << 20, None) == 1


def test_station_major_validation():
    """The station-major entry point takes complex float32 on the 64-station
    matrix-core kernel or the vector-ALU kernel, int8 and 16-bit samples on the
    64-station direct-to-LDS kernel, and rejects everything else before any
    launch."""
    lib = _lib.load()
    X, V = VP(1 << 20), VP(2 << 20)

    def call(cfg, in_type=0, S=70, P=2, C=3, T=50, x=X, v=V, out_type=0, acc=0):
        return lib.xc_correlate_station_major(ctypes.byref(cfg) if cfg else None, x, in_type, S, P, C, T, v,
                                              out_type, acc, None)

    unsupported, invalid = 2, 1
    # int8 and 16-bit: accepted (a null pointer then fails the argument check)
    assert call(None, in_type=xe.XC_IN_CI8, out_type=xe.XC_OUT_CI32, x=None) == invalid
    assert call(None, in_type=xe.XC_IN_CF16, x=None) == invalid
    # but not on the register-staged, 32-station or vector-ALU kernels
    assert call(_lib.XcConfig(xe.XC_KERNEL_MFMA, 64, 0, 0, xe.XC_STAGING_REGISTERS, 0), in_type=xe.XC_IN_CI8,
                out_type=xe.XC_OUT_CI32) == unsupported
    assert call(_lib.XcConfig(xe.XC_KERNEL_MFMA, 32, 0, 0, 0, 0), in_type=xe.XC_IN_CBF16) == unsupported
    assert call(_lib.XcConfig(xe.XC_KERNEL_VALU, 0, 0, 0, 0, 0), in_type=xe.XC_IN_CF16) == unsupported
    assert call(_lib.XcConfig(xe.XC_KERNEL_VALU, 0, 0, 0, 0, 0), x=None) == invalid   # VALU takes it
    assert call(_lib.XcConfig(xe.XC_KERNEL_MFMA, 32, 0, 0, 0, 0)) == unsupported
    assert call(None, P=3) == unsupported
    assert call(None, x=None) == invalid
    assert call(None, v=VP((2 << 20) + 8)) == invalid
    assert call(None, acc=2) == invalid
    assert call(None, T=0) == invalid
    # what it resolves to: the 64-station matrix-core kernel, at any station count
    for S in (1, 8, 48, 70):
        r = _lib.XcConfig()
        assert lib.xc_resolve_config(ctypes.byref(_lib.XcConfig(xe.XC_KERNEL_MFMA, 64, 0, 0, 0, 0)), 0, 0, S, 2, 3,
                                     50, ctypes.byref(r)) == 0
        assert (r.kernel, r.block) == (xe.XC_KERNEL_MFMA, 64)


def test_tune_candidates_pruned_by_table1():
    """The vector-ALU register tiles the tuner times are those of {2, 4, 8}^2
    (one of each mirror pair) whose Table 1 register count, plus staging and
    address registers, fits 256: 8 x 4, 4 x 8 and 8 x 8 are pruned."""
    cands = xe.tune_candidates(_lib.XC_IN_CF32)
    tiles = {(c["tile_w"], c["tile_h"]) for c in cands if c["kernel"] == _lib.XC_KERNEL_VALU and c["block"] == 32}
    assert tiles == {(4, 4), (8, 2), (4, 2), (2, 2)}
    for w, h in [(8, 4), (8, 8)]:
        assert xe.tile_cost(w, h)[2] > 256 - 24
    # and the one-channel kernel for arrays of at most 16 stations
    assert sum(1 for c in cands if c["kernel"] == _lib.XC_KERNEL_VALU and c["block"] == 16) == 1
    for c in cands:        # every candidate resolves for a small array
        r = xe.resolve_config((_lib.XC_IN_CF32, 4, 64, 12, 2), config=c)
        assert r["kernel"] == c["kernel"]
    i8 = xe.tune_candidates(_lib.XC_IN_CI8)
    assert all(c["kernel"] == _lib.XC_KERNEL_MFMA for c in i8) and len(i8) == 3


def test_small_array_kernel_resolution():
    # complex float32 on at most 16 stations: the one-channel kernel (vector ALU, block 16) by default
    r = xe.resolve_config((_lib.XC_IN_CF32, 16, 256, 8, 2))
    assert (r["kernel"], r["block"], r["time_chunk"], r["time_split"]) == (_lib.XC_KERNEL_VALU, 16, 128, 1)
    assert xe.resolve_config((_lib.XC_IN_CF32, 16, 256, 16, 2))["block"] == 16
    assert xe.resolve_config((_lib.XC_IN_CF32, 16, 256, 17, 2))["kernel"] == _lib.XC_KERNEL_MFMA
    assert xe.resolve_config((_lib.XC_IN_CI8, 16, 256, 8, 2), _lib.XC_OUT_CI32)["kernel"] == _lib.XC_KERNEL_MFMA
    # an explicit kernel choice keeps its own defaults
    assert xe.resolve_config((_lib.XC_IN_CF32, 16, 256, 8, 2), config={"kernel": _lib.XC_KERNEL_VALU})["block"] == 32
    assert xe.resolve_config((_lib.XC_IN_CF32, 16, 256, 8, 2), config={"kernel": _lib.XC_KERNEL_MFMA})["block"] == 32
    for bad in [dict(kernel=_lib.XC_KERNEL_VALU, block=16, tile_w=2, tile_h=2),
                dict(kernel=_lib.XC_KERNEL_VALU, block=16, time_chunk=32),
                dict(kernel=_lib.XC_KERNEL_VALU, block=16, time_split=2)]:
        with pytest.raises(xe.XengineError):
            xe.resolve_config((_lib.XC_IN_CF32, 16, 256, 8, 2), config=bad)
    with pytest.raises(xe.XengineError):      # at most 16 stations
        xe.resolve_config((_lib.XC_IN_CF32, 16, 256, 20, 2), config={"kernel": _lib.XC_KERNEL_VALU, "block": 16})


def test_tune_buckets():
    b = lambda S, C, T, it=_lib.XC_IN_CI8: xe.tune_bucket(it, _lib.XC_OUT_CI32 if it == 1 else 0, S, C, T)
    assert b(100, 500, 768) == b(120, 600, 700)          # same 32-station blocks, T and unit classes
    assert b(100, 500, 768) != b(130, 500, 768)          # another station-block count
    f = lambda S: b(S, 64, 768, _lib.XC_IN_CF32)
    assert f(8) == f(16) != f(17) == f(32)                 # at most 16 stations: the one-channel kernel's bucket
    assert b(100, 500, 768) != b(101, 500, 768)          # 101 stations are not whole int8 copy granules
    assert b(100, 500, 768) != b(100, 500, 2000)         # another integration-length class
    assert b(100, 8, 768) != b(100, 500, 768)            # few units against a full device
    assert b(100, 5000, 768) == b(100, 9000, 768)        # unit class capped
    assert b(8, 16, 256, 0)[3] == 1                      # complex float32 is always whole granules
    with pytest.raises(xe.XengineError):
        xe.tune_bucket(0, 0, 0, 1, 1)


def test_server_rejects_bad_stream_descriptions():
    lib = _lib.load()
    srv = ctypes.c_void_p()
    assert lib.xc_server_create(1 << 30, ctypes.byref(srv)) == 0
    sid = ctypes.c_int32()
    bad = [dict(blocks_per_fold=3, blocks_per_integration=8),          # not a multiple
           dict(ring_blocks=3, blocks_per_fold=2),                     # fewer than two folds of slots
           dict(staggered=3), dict(staggered=-1), dict(n_pol=1), dict(block_times=0),
           dict(acc_type=_lib.XC_OUT_CI32, block_times=512, blocks_per_integration=256)]   # int32 bound
    for kw in bad:
        a = dict(n_stations=8, n_channels=2, block_times=16, blocks_per_integration=4, blocks_per_fold=2,
                 ring_blocks=4, in_type=_lib.XC_IN_CI8, acc_type=_lib.XC_OUT_CI32, staggered=1, n_pol=2,
                 block_period_s=0.0)
        a.update(kw)
        d = _lib.XcStreamDesc(a["n_stations"], a["n_pol"], a["n_channels"], a["block_times"],
                              a["blocks_per_integration"], a["blocks_per_fold"], a["ring_blocks"], a["in_type"],
                              a["acc_type"], a["staggered"], a["block_period_s"])
        assert lib.xc_stream_open(srv, ctypes.byref(d), ctypes.byref(sid)) != 0, kw
    # fold order: 0 or 1 only; no stream to flush (1 = XC_ERR_INVALID_ARG)
    assert lib.xc_server_set_fold_order(None, 1) == 1
    assert lib.xc_server_set_fold_order(srv, 2) == 1
    assert lib.xc_server_set_fold_order(srv, 1) == 0 and lib.xc_server_set_fold_order(srv, 0) == 0
    assert lib.xc_stream_flush(srv, 0) == 1
    assert lib.xc_stream_flush(None, 0) == 1
    lib.xc_server_destroy(srv)


def test_xc_log_records_tune_cache_loads(tmp_path):
    """XC_LOG names a file: a tuning-cache load is logged there, one line; with
    XC_LOG unset nothing is written.  (A fresh process each time: the library
    reads XC_LOG once.)"""
    import subprocess
    import sys as _sys
    cache = tmp_path / "tune.jsonl"
    cache.write_text('{"in": 0, "out": 1, "sb": 2, "gran": 1, "tb": 10, "ub": 10, "kernel": 2, "block": 64, '
                     '"time_chunk": 0, "time_split": 2, "staging": 0, "product": 0, "tile_w": 0, "tile_h": 0, '
                     '"ms": 0.1, "S": 64, "C": 256, "T": 768}\n')
    code = ("import sys; sys.path.insert(0, %r); import paper_1702_00844_amd as xe; "
            "print(xe.tune_cache_load(%r))" % (os.path.dirname(os.path.dirname(os.path.abspath(__file__))), str(cache)))
    log = tmp_path / "xc.log"
    env = dict(os.environ, XC_LOG=str(log))
    out = subprocess.run([_sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    n = int(out.stdout.strip().splitlines()[-1])
    lines = log.read_text().splitlines()
    assert lines == ["[xengine] tune cache %s: %d entries loaded" % (cache, n)], lines
    env.pop("XC_LOG")
    log2 = tmp_path / "none.log"
    out = subprocess.run([_sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and not log2.exists() and "[xengine]" not in out.stderr


def test_kernel_source_hash_ignores_comments_and_layout():
    # bench.py reports counter-measured HBM traffic only while profiles/traffic.json
    # was taken on the same kernel code; comments and layout are not code
    import bench
    src = 'int a; // "x" note\n/* block\n   comment */ const char *s = "a // b \\" /* c */";\n  x  =  1;'
    assert bench.code_text(src) == 'int a; const char *s = "a // b \\" /* c */"; x = 1;'
    assert bench.code_text("x = 1; // one") == bench.code_text("x  =  1;\n")
    assert bench.code_text("x = 1;") != bench.code_text("x = 2;")
    assert bench.code_text("c = '/';  // slash") == "c = '/';"
    for kind in bench.KERNEL_SOURCES:
        assert len(bench.source_sha(kind)) == 16
