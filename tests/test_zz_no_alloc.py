"""GPU test of the allocation-free split entry point (xc_correlate_split_static):
two calls in a row, the second on a smaller input, each compared with the
workspace entry point (xc_correlate_split) on the same input and split, and
with the oracle."""
import numpy as np
import pytest
import torch

import paper_1702_00844_amd as xe
from paper_1702_00844_amd import _lib, inputs
from tests.helpers import gpu_vis_numpy, oracle_vis, rel_err

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("kind", ["cf32", "ci8"])
def test_static_scratch_matches_workspace_entry_point(kind):
    shapes = [(40, 12, 300, 7), (9, 3, 65, 4)]          # (S, C, T, split): the second call is smaller
    for S, C, T, split in shapes:
        if kind == "cf32":
            x = inputs.cn_gaussian(C, T, S, seed=S + T, device=DEV)
        else:
            x = inputs.ci8_gaussian(C, T, S, seed=S + T, device=DEV)
        ref_split = xe.correlate(x, split=split)
        got = torch.full_like(ref_split, 5)
        xe.correlate_into(x, got, split=split, static_scratch=True)
        torch.cuda.synchronize()
        g = gpu_vis_numpy(got)
        if kind == "ci8":
            assert np.array_equal(g, gpu_vis_numpy(ref_split))
            assert np.array_equal(g, oracle_vis(x))
        else:
            # the same kernels, pieces and fixed-order sum: the same bits
            assert torch.equal(got, ref_split)
            assert rel_err(g, oracle_vis(x)) <= 1e-5
        # accumulate mode adds onto what is there
        base = got.clone()
        xe.correlate_into(x, got, split=split, static_scratch=True, accumulate=True)
        torch.cuda.synchronize()
        if kind == "ci8":
            assert np.array_equal(gpu_vis_numpy(got), 2 * gpu_vis_numpy(base))
        else:
            assert rel_err(gpu_vis_numpy(got), 2 * gpu_vis_numpy(base)) <= 1e-6


def test_static_scratch_rejects_oversized_split():
    S, C, T = 64, 64, 64
    x = inputs.cn_gaussian(C, T, S, seed=3, device=DEV)
    out = torch.empty(xe.vis_shape(C, S, xe.XC_OUT_CF32), dtype=torch.complex64, device=DEV)
    need = 64 * C * (S * (S + 1) // 2) * 4 * 8
    assert need > _lib.XC_SPLIT_STATIC_SCRATCH_BYTES
    with pytest.raises(xe.XengineError) as e:
        xe.correlate_into(x, out, split=64, static_scratch=True)
    assert e.value.status_name == "XC_ERR_UNSUPPORTED"
