"""Independent library contexts on separate HIP streams, each driven from its
own host thread, give bit for bit the results of one context running the same
work in sequence: contexts share no device state (workspaces, work-item
arrays and profile records are per context) and every kernel reduces in a
fixed order.  The work per job is the whole path on a small problem with
paired and partitioned passes: factor (LU and UL, spikes), FP32 rSVD build,
FP32 Parareal.
"""
import threading

import numpy as np
import pytest
import torch

from paper_2508_08873_amd import inputs

pytestmark = pytest.mark.gpu


def _job(lrpr, ctx, P, om, u0, f, fsc):
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt,
                   store_mask=lrpr.STORE_F64 | lrpr.STORE_F32 | lrpr.STORE_MIRROR | lrpr.STORE_SPLIT |
                   lrpr.STORE_UL)
    coarse = ctx.rsvd_build([(F, P.k, P.p, om[s]) for s in range(P.N)], P.m, 1)
    out = ctx.parareal_solve(coarse, [F] * P.N, P.m, u0, f, fsc, tol=1e-6, fine_prec=1)
    res = (np.array(coarse.sigma), out["U"][0].cpu().numpy(), out["iters"][0])
    coarse.close()
    F.close()
    return res


def test_two_pipelines_match_sequential():
    from paper_2508_08873_amd import lrpr
    from paper_2508_08873_amd.lrpr import colmajor
    P = inputs.tiny2d(nx=121, N=4, m=4, k=12, p=4, T=1.0 / 8)
    jobs = []
    for seed in (1, 2, 3, 4):
        r = np.random.default_rng(seed)
        om = [colmajor(torch.from_numpy(r.standard_normal((P.n, P.k + P.p))).to("cuda", torch.float32))
              for _ in range(P.N)]
        u0 = colmajor(torch.from_numpy(P.u0() + 0.1 * r.standard_normal(P.n)).reshape(-1, 1).to("cuda"))
        f = colmajor(torch.from_numpy(P.source().reshape(-1, 1)).to("cuda"))
        fsc = torch.from_numpy(np.concatenate([P.fscale(s) for s in range(1, P.N + 1)])).to("cuda")
        jobs.append((om, u0, f, fsc))
    torch.cuda.synchronize()
    print("sequential reference", flush=True)
    ref_ctx = lrpr.Context(0)
    ref = [_job(lrpr, ref_ctx, P, *j) for j in jobs]
    torch.cuda.synchronize()
    print("two pipelines", flush=True)
    pipes = []
    for _ in range(2):
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            pipes.append((st, lrpr.Context(0)))
    torch.cuda.synchronize()
    got = [None] * len(jobs)
    errs = []

    def worker(i):
        st, ctx = pipes[i]
        try:
            with torch.cuda.stream(st):
                for j in range(i, len(jobs), 2):
                    got[j] = _job(lrpr, ctx, P, *jobs[j])
            st.synchronize()
        except Exception as ex:
            errs.append(ex)

    th = [threading.Thread(target=worker, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    assert not errs, errs
    for j, (a, b) in enumerate(zip(ref, got)):
        assert np.array_equal(a[0], b[0]), ("sigma", j)
        assert np.array_equal(a[1], b[1]), ("parareal iterate", j)
        assert a[2] == b[2], ("iterations", j)
    for _, c in pipes:
        c.close()
    ref_ctx.close()
