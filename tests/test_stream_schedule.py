"""The streaming server's fold schedule, checked on the host (no device).

A stream integrates its blocks in sub-intervals whose partial sums are added
into a resident result (the paper's Section 4.5 does the same with the Cell's
local store) while blocks arrive in real time (Section 1).  These tests replay
the server's own schedule for many descriptors and check what must hold for
any of them: each block of each channel is folded exactly once into its own
integration, each block's last fold is enqueued within k - 1 blocks of its
arrival (the per-block deadline k P), an integration is published only after
every channel has folded all of it, and spread ends give the device one
group's fold per block."""
import ctypes
import itertools

import pytest

import paper_1702_00844_amd as xe
from paper_1702_00844_amd import _lib


def _desc(C, k, bpi, mode, S=8, bt=16):
    d = xe.Server.desc(S, C, bt, bpi, blocks_per_fold=k, staggered=mode > 0, spread_ends=mode == 2)
    return d


def _groups(C, k, mode):
    G = k if mode else 1
    return [(C * g // G, C * (g + 1) // G) for g in range(G)]


CASES = [(C, k, mult, mode, n, flush)
         for C, k, mult, mode in itertools.product([1, 3, 10], [1, 2, 3, 4, 6], [1, 2, 3], [0, 1, 2])
         for n, flush in [(0, False), (k * mult * 2, False), (k * mult * 2 + k + 1, False),
                          (k * mult * 3 - 1, True), (k * mult * 2 + 1, True)]]


@pytest.mark.parametrize("C,k,mult,mode,n,flush", CASES,
                         ids=["C%d_k%d_bpi%d_mode%d_n%d_f%d" % (c[0], c[1], c[1] * c[2], c[3], c[4], c[5])
                              for c in CASES])
def test_schedule_invariants(C, k, mult, mode, n, flush):
    bpi = k * mult
    d = _desc(C, k, bpi, mode)
    folds, pub = xe.Server.schedule(d, n, flush=flush)
    groups = _groups(C, k, mode)
    covered = [0] * len(groups)        # each group's first block not yet folded
    fold_of = {}                       # (group, block) -> trigger
    for trig, g, c0, c1, first, last in folds:
        assert 0 <= g < len(groups) and (c0, c1) == groups[g]
        assert first <= last <= trig <= max(n - 1, 0)           # only committed blocks are folded
        assert first // bpi == last // bpi                      # within one integration
        assert first == covered[g], (g, first, covered[g])      # in order, no gap, no block twice
        covered[g] = last + 1
        for b in range(first, last + 1):
            fold_of[(g, b)] = trig
    complete = n // bpi * bpi
    for g in range(len(groups)):
        if mode == 2 and not flush:
            # spread ends: a group folds what it has at its turn, every k blocks
            assert covered[g] >= max(0, n - k), (g, covered[g])
        else:
            assert covered[g] >= complete, (g, covered[g], complete)
        if mode == 0:
            assert covered[g] == n // k * k
    # the per-block deadline: a block's fold comes within k - 1 blocks of it
    # (the flush too: a block it folds would have come at its group's next turn, after the last commit)
    for (g, b), trig in fold_of.items():
        assert trig <= b + k - 1, (g, b, trig)
    # publication: in order, and only once every group has folded the whole integration
    n_int = n // bpi + 1
    assert len(pub) == n_int
    last_pub = -1
    for j, when in enumerate(pub):
        end = (j + 1) * bpi
        if when < 0:
            assert end > n or (mode == 2 and not flush), (j, when)
            continue
        assert when >= last_pub
        last_pub = when
        assert end <= n
        for g in range(len(groups)):
            t = fold_of[(g, end - 1)]
            assert t <= when, (j, g, t, when)
        if mode != 2:
            assert when == end - 1                      # at the integration's last block
        elif when < n:
            assert when <= end - 1 + max(k - 1, 0)      # k - 2 blocks into the next one, at most
    # an integration that every group has folded is published (by a commit or the flush)
    for j in range(n_int):
        end = (j + 1) * bpi
        if end <= n and all(covered[g] >= end for g in range(len(groups))):
            assert pub[j] >= 0, j
    # spread ends: one group's turn per block (its fold split at most once, at an integration end)
    if mode == 2:
        per_trigger = {}
        for trig, g, *_ in folds:
            if trig < n - 1 or not flush:
                per_trigger.setdefault(trig, set()).add(g)
        assert all(len(gs) == 1 for gs in per_trigger.values())


def test_schedule_worked_example():
    """10 channels in 4 groups (2, 3, 2 and 3 channels), 8 blocks per
    integration, folds of 4, spread ends: group m mod 4 folds at block m; at
    block 8 group 0 folds the rest of integration 0 (blocks 5-7) and block 8
    of integration 1 as two folds.  Integration 0 is complete once every group
    has folded through block 7: group 3 at block 7, group 0 at 8, group 1 at 9
    and group 2 at 10, so it is published after block 10 (k - 2 blocks into
    the next integration); integration 1 after block 18; the partial third
    one is not, even by the flush."""
    d = _desc(10, 4, 8, 2)
    folds, pub = xe.Server.schedule(d, 20, flush=True)
    assert folds[:12] == [
        (0, 0, 0, 2, 0, 0), (1, 1, 2, 5, 0, 1), (2, 2, 5, 7, 0, 2), (3, 3, 7, 10, 0, 3),
        (4, 0, 0, 2, 1, 4), (5, 1, 2, 5, 2, 5), (6, 2, 5, 7, 3, 6), (7, 3, 7, 10, 4, 7),
        (8, 0, 0, 2, 5, 7), (8, 0, 0, 2, 8, 8), (9, 1, 2, 5, 6, 7), (9, 1, 2, 5, 8, 9)]
    assert pub == [10, 18, -1]
    # without spread ends every group folds its remainder at block 7
    folds1, pub1 = xe.Server.schedule(_desc(10, 4, 8, 1), 8)
    assert [f for f in folds1 if f[0] == 7] == [(7, 3, 7, 10, 4, 7), (7, 0, 0, 2, 5, 7), (7, 1, 2, 5, 6, 7),
                                                (7, 2, 5, 7, 7, 7)]
    assert pub1 == [7, -1]


def test_schedule_errors():
    d = _desc(4, 2, 4, 1)
    n = ctypes.c_int64()
    lib = xe.lib()
    assert lib.xc_stream_schedule(ctypes.byref(d), 4, 0, None, 0, None, None, 0) == 1
    assert lib.xc_stream_schedule(ctypes.byref(d), -1, 0, None, 0, ctypes.byref(n), None, 0) == 1
    assert lib.xc_stream_schedule(ctypes.byref(d), 4, 2, None, 0, ctypes.byref(n), None, 0) == 1
    assert lib.xc_stream_schedule(ctypes.byref(d), 4, 0, None, 3, ctypes.byref(n), None, 0) == 1
    assert lib.xc_stream_schedule(None, 4, 0, None, 0, ctypes.byref(n), None, 0) == 1
    bad = _desc(4, 3, 4, 1)                     # 4 blocks per integration, folds of 3
    assert lib.xc_stream_schedule(ctypes.byref(bad), 4, 0, None, 0, ctypes.byref(n), None, 0) == 1
    bad = _desc(4, 2, 4, 1)
    bad.staggered = 3
    assert lib.xc_stream_schedule(ctypes.byref(bad), 4, 0, None, 0, ctypes.byref(n), None, 0) == 1
    # counting only: the folds are counted past max_folds.  Two groups, 4
    # blocks per integration: one fold per block, and at an integration's last
    # block the other group's remainder too, 5 per integration
    assert lib.xc_stream_schedule(ctypes.byref(d), 8, 0, None, 0, ctypes.byref(n), None, 0) == 0
    assert n.value == 10
