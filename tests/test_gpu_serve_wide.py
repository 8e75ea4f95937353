"""GPU tests of the serving loop on the factors the serving benchmark uses.

The serving operators keep FP64 tiles, the mirrored set and the spikes of the
partitioned substitution.  Ten requests of the 127^2 serving operator (64
slices x 32 steps, k = 48, p = 12) are submitted together, so one fine sweep
carries 10 x 64 columns = 40 sixteen-column groups: more than the width up to
which a plain batched sweep takes the partitioned passes.  The checks:

* every request's result is the same bit for bit alone and in the mix;
* served results equal the oracle's sequential fine solution
  u_n = F_n u_{n-1} (the fixed point of the Parareal iteration of eq.
  def_Parareal, reached to tolerance 1e-12) to 1e-11 relative, on sampled
  requests;
* the same ten problems through lrpr_parareal_solve (nreq = 10) equal the
  served results and each problem solved alone.
"""
import numpy as np
import pytest
import torch

from paper_2508_08873_amd import inputs

pytestmark = pytest.mark.gpu

NREQ = 10
TOL = 1e-12


def _dev(a):
    from paper_2508_08873_amd.lrpr import colmajor
    a = np.ascontiguousarray(a)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    return colmajor(torch.from_numpy(a).to("cuda", torch.float64))


@pytest.fixture(scope="module")
def op127():
    from paper_2508_08873_amd import lrpr
    ctx = lrpr.Context(0)
    P = inputs.serve3()[0]
    assert P.nx == 127
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt,
                   store_mask=lrpr.STORE_F64 | lrpr.STORE_MIRROR | lrpr.STORE_SPLIT)
    Om = torch.empty((P.N, P.l, P.n), dtype=torch.float64, device="cuda")
    ctx.randn(Om, 7, 127)
    coarse = ctx.rsvd_build([(F, P.k, P.p, Om[s].t()) for s in range(P.N)], P.m, 0)
    del Om
    fsc = torch.from_numpy(np.concatenate([P.fscale(s) for s in range(1, P.N + 1)])).to("cuda")
    reqs = [(P.u0(req=i + 1), P.source(req=i + 1)) for i in range(NREQ)]
    yield {"ctx": ctx, "P": P, "F": F, "coarse": coarse, "fsc": fsc, "reqs": reqs}
    coarse.close()
    F.close()
    ctx.close()


def _serve(o, idx):
    """Serve the requests idx, all submitted before the first step; returns
    {i: (U host (N+1) x n, iterations)}."""
    from paper_2508_08873_amd import lrpr
    P = o["P"]
    srv = lrpr.Server(o["ctx"], [(o["coarse"], [o["F"]] * P.N, P.m, o["fsc"])], tol=TOL, budget_bytes=1 << 36)
    ids = {}
    for i in idx:
        u0, f = o["reqs"][i]
        rid, U = srv.submit(0, _dev(u0), _dev(f))
        ids[rid] = (i, U)
    done, steps = {}, 0
    peak = 0
    while len(done) < len(idx):
        fin = srv.progress(wait=True)
        peak = max(peak, srv.stats()["active"] + len(fin))
        steps += 1
        for rid, it in fin:
            i, U = ids[rid]
            done[i] = (U.t().cpu().numpy().copy(), it)
        assert steps < 200
    srv.close()
    return done, peak


def test_serve_wide_spike_factors_alone_vs_mix(op127, ora):
    o = op127
    P = o["P"]
    mix, peak = _serve(o, list(range(NREQ)))
    # every request was in the first step: 40 column groups in one sweep
    assert peak == NREQ
    for i in range(NREQ):
        alone, _ = _serve(o, [i])
        assert alone[i][1] == mix[i][1]
        assert np.array_equal(alone[i][0], mix[i][0]), "request %d differs alone vs in the mix" % i
    # sampled requests against the oracle's sequential fine solution
    sample = [0, 3, 9]
    op = ora.Operator(**P.op_params())
    X = np.stack([o["reqs"][i][0] for i in sample], axis=1)
    f = np.stack([o["reqs"][i][1] for i in sample], axis=1)
    fcol = np.arange(len(sample), dtype=np.int32)
    seq = [X]
    for s in range(1, P.N + 1):
        seq.append(op.fine(seq[-1], P.m, f, fcol, np.tile(P.fscale(s), (len(sample), 1))))
    seq = np.stack(seq)   # (N+1) x n x len(sample)
    for j, i in enumerate(sample):
        ref = seq[:, :, j]
        err = np.linalg.norm(mix[i][0] - ref, axis=1).max() / np.linalg.norm(ref, axis=1).max()
        print("request %d: %d iterations, relative error vs sequential fine solution %.2e" % (i, mix[i][1], err))
        assert err <= 1e-11


def test_parareal_solve_wide_equals_served(op127):
    o = op127
    P = o["P"]
    ctx = o["ctx"]
    u0 = np.stack([r[0] for r in o["reqs"]], axis=1)
    f = np.stack([r[1] for r in o["reqs"]], axis=1)
    out = ctx.parareal_solve(o["coarse"], [o["F"]] * P.N, P.m, _dev(u0), _dev(f), o["fsc"], tol=TOL)
    assert out["status"] == 0
    served, _ = _serve(o, [1, 4])
    for i in (1, 4):
        alone = ctx.parareal_solve(o["coarse"], [o["F"]] * P.N, P.m, _dev(u0[:, i]), _dev(f[:, i]), o["fsc"],
                                   tol=TOL)
        assert alone["iters"][0] == out["iters"][i] == served[i][1]
        a = alone["U"][0].cpu().numpy()
        assert np.array_equal(a, out["U"][i].cpu().numpy()), "problem %d differs alone vs with nreq=10" % i
        assert np.abs(served[i][0] - a).max() <= 1e-14 * np.abs(a).max()
