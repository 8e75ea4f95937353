"""GPU test of lrpr_coarse_apply_noalloc, the coarse apply for callers that
cannot allocate device memory: through the C ABI, two calls in a row (the
second on a smaller input: fewer columns of a smaller operator's slice)
equal lrpr_coarse_apply bit for bit, and a call whose scratch would exceed
the fixed array is refused with LRPR_ERR_ARG."""
import numpy as np
import pytest
import torch

from paper_2508_08873_amd import inputs

pytestmark = pytest.mark.gpu


def _build(ctx, P, seed):
    from paper_2508_08873_amd import lrpr
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt, store_mask=lrpr.STORE_F64)
    Om = torch.empty((P.N, P.l, P.n), dtype=torch.float64, device="cuda")
    ctx.randn(Om, seed, 0)
    coarse = ctx.rsvd_build([(F, P.k, P.p, Om[s].t()) for s in range(P.N)], P.m, 0)
    return F, coarse


def test_coarse_apply_noalloc_matches_apply():
    from paper_2508_08873_amd import lrpr
    ctx = lrpr.Context(0)
    big = inputs.dar255(N=3, m=4)
    small = inputs.tiny2d(nx=31, N=4, m=4, k=8, p=3)
    Fb, Cb = _build(ctx, big, 1)
    Fs, Cs = _build(ctx, small, 2)
    cases = [(Cb, 2, big.n, 64), (Cs, 1, small.n, 5)]
    for coarse, s, n, w in cases:
        X = lrpr.colmajor(torch.from_numpy(np.random.default_rng([n, w]).standard_normal((n, w))).to("cuda"))
        want = coarse.apply(s, X)
        out = torch.full_like(X, np.nan)
        got = coarse.apply_noalloc(s, X, out)
        torch.cuda.synchronize()
        print("noalloc apply n=%d w=%d: max |diff| %.3e" % (n, w, (got - want).abs().max().item()), flush=True)
        assert torch.equal(got, want)
        assert torch.isfinite(got).all()
    # scratch limit: (ceil(n/256) + 1) * k * min(w, 12288/k) doubles above 16 MiB
    X = lrpr.colmajor(torch.zeros((big.n, 1024), dtype=torch.float64, device="cuda"))
    with pytest.raises(lrpr.LrprError) as ei:
        Cb.apply_noalloc(0, X)
    assert ei.value.status == 1
    Cb.close()
    Cs.close()
    Fb.close()
    Fs.close()
    ctx.close()
