"""GPU check of the on-device Gaussian generator (lrpr_randn) against the
test-side Philox4x32-10 + Box-Muller reference (oracle/philox.py, pinned to
the generator's published known-answer vectors): the integer stream must be
the same, so FP64 values agree to the rounding of log / sqrt / cos / sin, and
FP32 values are the FP64 ones rounded once."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2508_08873_amd import lrpr
    return lrpr.Context(0)


@pytest.mark.parametrize("count,seed,stream", [(1, 0, 0), (7, 5, 1), (4096, 2024, 3), (100001, (7 << 40) + 9, 2**33 + 1)])
def test_randn_matches_reference(ctx, count, seed, stream):
    from oracle import philox
    ref = philox.randn(count, seed, stream)
    X = ctx.randn(torch.empty(count, dtype=torch.float64, device="cuda"), seed, stream)
    got = X.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    X32 = ctx.randn(torch.empty(count, dtype=torch.float32, device="cuda"), seed, stream)
    assert np.abs(X32.cpu().numpy().astype(np.float64) - ref).max() <= 1e-6 * max(1.0, np.abs(ref).max())


def test_randn_slices_are_independent_draws(ctx):
    """Streams differ, a prefix of a draw equals the shorter draw, moments of a large draw."""
    a = ctx.randn(torch.empty(1 << 20, dtype=torch.float64, device="cuda"), 1, 0)
    b = ctx.randn(torch.empty(1 << 20, dtype=torch.float64, device="cuda"), 1, 1)
    c = ctx.randn(torch.empty(1000, dtype=torch.float64, device="cuda"), 1, 0)
    assert torch.equal(a[:1000], c)
    assert not torch.equal(a[:1000], b[:1000])
    n = a.numel()
    assert abs(a.mean().item()) < 5.0 / n ** 0.5
    assert abs(a.var().item() - 1.0) < 5.0 * (2.0 / n) ** 0.5
