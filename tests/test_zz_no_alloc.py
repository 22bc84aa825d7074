"""The allocation-free entry point fmc_rrf_rms_noalloc against fmc_rrf_rms.

Both run the same kernel on the same inputs; the allocation-free one reads
the weights from the library's static per-device scratch instead of a buffer
of the context.  Two calls in a row, the second with a smaller input (fewer
trajectories, fewer steps and fewer variables), so that the second call
must not see anything of the first in the shared scratch.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def test_noalloc_matches_allocating_entry_point(fmc):
    import torch
    ctx = fmc.Context(0)
    rng = np.random.default_rng(17)
    for n, S, V in ((300, 777, 23), (37, 100, 5)):
        traj = torch.tensor(rng.normal(size=(n, S + 1, V)), dtype=torch.float64, device="cuda")
        w = rng.normal(size=V)
        ref = ctx.rrf_rms(traj, w, 0.005).cpu().numpy()
        out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        got = ctx.rrf_rms_noalloc(traj, w, 0.005, out).cpu().numpy()
        assert np.array_equal(got, ref), (n, S, V)
        # and the oracle's definition (trapezoid RMS), to its FP64 rounding
        o = oracle.rrf_rms(traj.cpu().numpy(), w, 0.005)
        np.testing.assert_allclose(got, o, rtol=1e-12, atol=0)
    with pytest.raises(fmc.FmcError) as e:  # beyond the static scratch
        ctx.rrf_rms_noalloc(torch.zeros((1, 2, 2049), dtype=torch.float64, device="cuda"),
                            np.ones(2049), 0.1, torch.empty(1, dtype=torch.float64, device="cuda"))
    assert e.value.code == fmc.EINVAL
    ctx.close()
