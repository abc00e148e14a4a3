"""The oracle against what the correlation definition fixes (CPU only)."""
import numpy as np
import pytest

import oracle
from tests import oracle_pins as pins


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda f: f.__name__)
def test_oracle_pin(check):
    check(oracle.load())


def test_point_source_stack():
    """Noise plus three point sources (the LOFAR-scale workload's recipe, at a
    reduced channel count): phase-referencing every cross-correlation to one
    source and averaging recovers that source's power A^2 = 0.01; the noise of
    the average is about 1/sqrt(T * baselines * channels * pols)."""
    from paper_1702_00844_amd import inputs
    C, T, S = 24, 768, 32
    x, prm = inputs.point_sources(C, T, S, seed=2)
    vis = oracle.correlate_f64(x.numpy())
    ph = prm["phase"]                       # [K, C, S]
    i_idx, j_idx = np.triu_indices(S, k=1)  # i < j
    bl = j_idx * (j_idx + 1) // 2 + i_idx
    n_stack = C * len(bl) * 2
    noise = 1.0 / np.sqrt(T * n_stack)
    for k in range(ph.shape[0]):
        ref = np.exp(-1j * (ph[k][:, i_idx] - ph[k][:, j_idx]))     # [C, nb]
        stack = 0
        for p in range(2):
            stack = stack + np.sum(vis[:, bl, p, p] * ref)
        est = stack / (n_stack * T)
        assert abs(est - prm["amplitude"] ** 2) < 6 * noise + 3e-4, (k, est)
    # a wrong conjugation (phase referenced the other way) recovers nothing
    ref = np.exp(+1j * (ph[0][:, i_idx] - ph[0][:, j_idx]))
    bad = np.sum(vis[:, bl, 0, 0] * ref) / (C * len(bl) * T)
    assert abs(bad) < 0.2 * prm["amplitude"] ** 2


def test_baseline_numbering():
    # b(i,j) enumerates pairs in the order of the reference loop nest
    # (station2 outer, station1 <= station2 inner) without gaps.
    order = [(i, j) for j in range(9) for i in range(j + 1)]
    assert [oracle.baseline_index(i, j) for i, j in order] == list(range(len(order)))
    assert oracle.n_baselines(64) == 2080 and oracle.n_baselines(256) == 32896
