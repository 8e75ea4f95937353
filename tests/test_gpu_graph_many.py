"""GPU tests of the graph-captured Parareal iteration and of several uneven
problems solved together (lrpr_parareal_solve_many).

* graph replay vs eager launches: with LRPR_TUNE_PARAREAL_GRAPH = 1 a
  Parareal iteration is captured once and replayed; the iterates and
  increments equal those of kernel-by-kernel launches (0) bit for bit after
  every replay count tried (max_iter = 1, 2, 3 and to convergence), with
  the host's reads of the increments, its convergence checks and the
  upload of the active flags between replays; FP64 and FP32 fine solves,
  plain and partitioned (spike) factors, two requests;
* four problems of different grids, slice counts, ranks and request
  counts in one call: each problem's result equals the same problem solved
  alone, bit for bit, and the oracle's Parareal (own rSVD on the same
  Omega) to 1e-11 with the same iteration count.
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
    c.tune_set(lrpr.TUNE_PARAREAL_GRAPH, 1)
    c.close()


def _dev(a):
    from paper_2508_08873_amd.lrpr import colmajor
    a = np.ascontiguousarray(a)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    return colmajor(torch.from_numpy(a).to("cuda", torch.float64))


def _setup(ctx, P, mask, prec):
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt, store_mask=mask)
    oms = [P.omega(s) for s in range(1, P.N + 1)]
    dt = torch.float64 if prec == 0 else torch.float32
    coarse = ctx.rsvd_build([(F, P.k, P.p, _dev(oms[s]).to(dt)) for s in range(P.N)], P.m, prec)
    fsc = torch.from_numpy(np.concatenate([P.fscale(s) for s in range(1, P.N + 1)])).to("cuda")
    return F, coarse, oms, fsc


@pytest.mark.parametrize("prec,split", [(0, False), (0, True), (1, True)], ids=["f64", "f64_split", "f32_split"])
def test_graph_replay_equals_eager(ctx, prec, split):
    from paper_2508_08873_amd import lrpr
    P = inputs.tiny2d(nx=31, N=6, m=4, k=6, p=3, tol=1e-13)
    mask = (lrpr.STORE_F64 if prec == 0 else lrpr.STORE_F32 | lrpr.STORE_F64) | lrpr.STORE_MIRROR
    mask |= lrpr.STORE_SPLIT if split else 0
    F, coarse, _, fsc = _setup(ctx, P, mask, prec)
    u0 = _dev(np.stack([P.u0(req=r) for r in range(2)], axis=1))
    f = _dev(np.stack([P.source(req=r) for r in range(2)], axis=1))
    for mi in (1, 2, 3, None):
        outs = []
        for graph in (0, 1):
            ctx.tune_set(lrpr.TUNE_PARAREAL_GRAPH, graph)
            o = ctx.parareal_solve(coarse, [F] * P.N, P.m, u0, f, fsc, tol=1e-13 if prec == 0 else 1e-6,
                                   max_iter=mi, fine_prec=prec)
            torch.cuda.synchronize()
            outs.append((o["U"].cpu().numpy(), o["iters"], o["incr"], o["status"]))
        (Ue, ie, ince, se), (Ug, ig, incg, sg) = outs
        assert ie == ig and se == sg and ince == incg, (mi, ie, ig)
        assert np.array_equal(Ue, Ug), "graph replay differs from eager launches, max_iter %s" % mi
    ctx.tune_set(lrpr.TUNE_PARAREAL_GRAPH, 1)
    coarse.close()
    F.close()


def _problems():
    return [inputs.tiny2d(nx=15, N=5, m=4, k=5, p=3, tol=1e-12, pid=11),
            inputs.tiny2d(nx=31, N=8, m=4, k=8, p=2, tol=1e-12, beta=(-5.0, 12.0), pid=12),
            inputs.tiny2d(nx=24, N=3, m=4, k=6, p=4, tol=1e-12, nu=0.7, c=3.0, pid=13),
            inputs.tiny2d(nx=40, N=6, m=4, k=10, p=4, tol=1e-12, beta=(0.0, 25.0), pid=14)]


def test_uneven_problems_together(ctx, ora):
    from paper_2508_08873_amd import lrpr
    nreqs = [1, 2, 1, 3]
    probs, ref = [], []
    for P, nr in zip(_problems(), nreqs):
        F, coarse, oms, fsc = _setup(ctx, P, lrpr.STORE_F64 | lrpr.STORE_MIRROR | lrpr.STORE_SPLIT, 0)
        u0 = np.stack([P.u0(req=r) for r in range(nr)], axis=1)
        f = np.stack([P.source(req=r) for r in range(nr)], axis=1)
        probs.append({"coarse": coarse, "factors": [F] * P.N, "u0": _dev(u0), "f": _dev(f), "fscale": fsc,
                      "tol": P.tol, "_P": P, "_F": F, "_oms": oms, "_u0": u0, "_f": f})
    together = ctx.parareal_solve_many(probs, nsteps=4)
    for i, pr in enumerate(probs):
        P = pr["_P"]
        alone = ctx.parareal_solve_many([pr], nsteps=4)[0]
        assert together[i]["status"] == 0
        assert alone["iters"] == together[i]["iters"]
        assert np.array_equal(alone["U"].cpu().numpy(), together[i]["U"].cpu().numpy()), "problem %d" % i
        single = ctx.parareal_solve(pr["coarse"], pr["factors"], P.m, pr["u0"], pr["f"], pr["fscale"], tol=P.tol)
        assert np.array_equal(single["U"].cpu().numpy(), together[i]["U"].cpu().numpy())
        op = ora.Operator(**P.op_params())
        for r in range(pr["u0"].shape[1]):
            sl = [ora.Slice(op, P.m, pr["_f"][:, r], P.fscale(s)) for s in range(1, P.N + 1)]
            ora.build_coarse(sl, P.k, P.p, pr["_oms"])
            o = ora.parareal(sl, pr["_u0"][:, r], tol=P.tol)
            Uo = o["iterates"][-1]
            Ug = together[i]["U"][r].cpu().numpy()
            err = np.linalg.norm(Ug - Uo, axis=1).max() / np.linalg.norm(Uo, axis=1).max()
            assert o["iters"] == together[i]["iters"][r], (i, r)
            assert err <= 1e-11, (i, r, err)
    for pr in probs:
        pr["coarse"].close()
        pr["_F"].close()
