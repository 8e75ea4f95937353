"""rSVD builds split into chunks by the panel budget, and coarse views.

No step of the build couples slices, so a build done in chunks must give
every slice the same singular values and coarse factors, bit for bit, as
the build of all slices at once; a view of slices [first, first+count)
must hand out exactly those slices' arrays, and Parareal on a view must
equal Parareal on a handle built from those slices alone.
"""
import numpy as np
import pytest
import torch

from paper_2508_08873_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2508_08873_amd import lrpr
    c = lrpr.Context(0)
    yield c
    c.tune_set(lrpr.TUNE_RSVD_BUDGET, 0)


def _slices(ctx, lrpr, probs, prec):
    """Slices of several problems of different grids, each with its own
    factor and Philox test matrices."""
    out, facs = [], []
    for i, P in enumerate(probs):
        F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt, store_mask=lrpr.STORE_F64 | lrpr.STORE_F32)
        facs.append(F)
        dt = torch.float32 if prec == 1 else torch.float64
        for s in range(P.N):
            Om = torch.empty((P.l, P.n), device="cuda", dtype=dt)
            ctx.randn(Om, 5, 100 * i + s)
            out.append((F, P.k, P.p, Om.t()))
    return out, facs


def _arrays(coarse, s):
    from paper_2508_08873_amd.lrpr import device_view
    k, n, U, S, V = coarse.get(s)
    torch.cuda.synchronize()
    return (device_view(U, n, k).cpu().clone(), device_view(S, k, 1).cpu().clone(),
            device_view(V, n, k).cpu().clone())


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_chunked_build_equals_one_build(ctx, prec):
    from paper_2508_08873_amd import lrpr
    probs = [inputs.tiny2d(nx=31, N=3, m=4, k=6, p=3), inputs.tiny2d(nx=47, N=4, m=4, k=9, p=2, beta=(3.0, -8.0)),
             inputs.tiny2d(nx=23, N=2, m=4, k=5, p=3)]
    slices, facs = _slices(ctx, lrpr, probs, prec)
    ctx.tune_set(lrpr.TUNE_RSVD_BUDGET, 0)
    whole = ctx.rsvd_build(slices, 4, prec)
    # a budget below two slices' panels: chunks of one slice each
    ctx.tune_set(lrpr.TUNE_RSVD_BUDGET, 1)
    parts = ctx.rsvd_build(slices, 4, prec)
    ctx.tune_set(lrpr.TUNE_RSVD_BUDGET, 0)
    assert whole.sigma == parts.sigma
    assert whole.fallback == parts.fallback
    for s in range(len(slices)):
        for a, b in zip(_arrays(whole, s), _arrays(parts, s)):
            assert torch.equal(a, b), s
    whole.close()
    parts.close()
    for F in facs:
        F.close()


def test_view_slices_and_parareal(ctx):
    from paper_2508_08873_amd import lrpr
    probs = [inputs.tiny2d(nx=31, N=3, m=4, k=6, p=3), inputs.tiny2d(nx=47, N=4, m=4, k=9, p=2, beta=(3.0, -8.0))]
    slices, facs = _slices(ctx, lrpr, probs, 0)
    allc = ctx.rsvd_build(slices, 4, 0)
    alone = ctx.rsvd_build(slices[3:], 4, 0)
    v = allc.view(3, 4)
    assert v.sigma == alone.sigma
    for s in range(4):
        for a, b in zip(_arrays(v, s), _arrays(allc, 3 + s)):
            assert torch.equal(a, b)
    P = probs[1]
    u0 = lrpr.colmajor(torch.from_numpy(P.u0().reshape(-1, 1)).to("cuda"))
    f = lrpr.colmajor(torch.from_numpy(P.source().reshape(-1, 1)).to("cuda"))
    fsc = torch.from_numpy(np.concatenate([P.fscale(s) for s in range(1, P.N + 1)])).to("cuda")
    outs = []
    for c in (v, alone):
        o = ctx.parareal_solve_many([{"coarse": c, "factors": [facs[1]] * P.N, "u0": u0, "f": f, "fscale": fsc,
                                      "tol": 1e-10}], P.m, fine_prec=0)[0]
        outs.append(o)
    assert outs[0]["iters"] == outs[1]["iters"]
    assert torch.equal(outs[0]["U"], outs[1]["U"])
    assert outs[0]["apost"] == outs[1]["apost"]
    with pytest.raises(lrpr.LrprError):
        allc.view(5, 3)
    v.close()
    alone.close()
    allc.close()
    for F in facs:
        F.close()
