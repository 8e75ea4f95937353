"""GPU tests of the serving loop (continuous batching of Parareal solves).

* every request's converged iterate equals the oracle's Parareal iterate for
  the same u0 and f (1e-11 relative, same iteration count);
* a request's result is bit-identical alone and in a mix of requests of two
  operators that arrive while other requests are on the GPU;
* admission by byte budget bounds the requests in flight, and all of them
  still complete with the same results;
* a served request equals lrpr_parareal_solve on the same input.
"""
import numpy as np
import pytest
import torch

from paper_2508_08873_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2508_08873_amd import lrpr
    return lrpr.Context(0)


def _dev(a):
    from paper_2508_08873_amd.lrpr import colmajor
    return colmajor(torch.from_numpy(np.ascontiguousarray(a)).to("cuda", torch.float64))


def _problems():
    return [inputs.tiny2d(nx=31, N=6, m=4, k=8, p=3, tol=1e-12),
            inputs.tiny2d(nx=23, N=5, m=3, k=6, p=2, beta=(-6.0, 14.0), tol=1e-12, pid=7)]


@pytest.fixture(scope="module")
def setup(ctx):
    from paper_2508_08873_amd import lrpr
    ops = []
    for P in _problems():
        F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt, store_mask=lrpr.STORE_F64 | lrpr.STORE_MIRROR)
        oms = [P.omega(s) for s in range(1, P.N + 1)]
        dev_oms = [_dev(o) for o in oms]
        coarse = ctx.rsvd_build([(F, P.k, P.p, dev_oms[s]) for s in range(P.N)], P.m, 0)
        fsc = torch.from_numpy(np.concatenate([P.fscale(s) for s in range(1, P.N + 1)])).to("cuda")
        ops.append({"P": P, "F": F, "coarse": coarse, "oms": oms, "fsc": fsc})
    return ops


def _server(ctx, setup, budget=1 << 34, max_active=0):
    from paper_2508_08873_amd import lrpr
    return lrpr.Server(ctx, [(o["coarse"], [o["F"]] * o["P"].N, o["P"].m, o["fsc"]) for o in setup],
                       tol=1e-12, budget_bytes=budget, max_active=max_active)


def _requests():
    """(op, u0, f) for 7 requests over the two operators."""
    out = []
    for i, (op, req) in enumerate([(0, 0), (1, 0), (0, 1), (0, 2), (1, 1), (0, 3), (1, 2)]):
        P = _problems()[op]
        out.append((op, P.u0(req=req), P.source(req=req)))
    return out


def _run(srv, reqs, arrive_at):
    """Submit request i once `arrive_at[i]` server steps have completed;
    return {i: (U host, iters)}."""
    done, ids, steps = {}, {}, 0
    pending = list(range(len(reqs)))
    while len(done) < len(reqs):
        for i in [j for j in pending if arrive_at[j] <= steps]:
            op, u0, f = reqs[i]
            rid, U = srv.submit(op, _dev(u0), _dev(f))
            ids[rid] = (i, U)
            pending.remove(i)
        fin = srv.progress(wait=True)
        steps += 1
        for rid, it in fin:
            i, U = ids[rid]
            done[i] = (U.cpu().numpy().copy(), it)
        assert steps < 200
    return done


def test_serve_matches_oracle_and_alone_vs_mix(ctx, ora, setup):
    reqs = _requests()
    srv = _server(ctx, setup)
    mix = _run(srv, reqs, arrive_at=[0, 0, 1, 1, 2, 3, 5])
    srv.close()
    for i, (op, u0, f) in enumerate(reqs):
        # alone, on a fresh server
        s1 = _server(ctx, setup)
        alone = _run(s1, [reqs[i]], arrive_at=[0])[0]
        s1.close()
        assert alone[1] == mix[i][1]
        assert np.array_equal(alone[0], mix[i][0]), "request %d differs alone vs in the mix" % i
        # oracle Parareal with its own rSVD of the same Omega
        o = setup[op]
        P = o["P"]
        opr = ora.Operator(**P.op_params())
        sl = [ora.Slice(opr, P.m, f, P.fscale(s)) for s in range(1, P.N + 1)]
        ora.build_coarse(sl, P.k, P.p, o["oms"])
        ref = ora.parareal(sl, u0, tol=1e-12)
        Uo = ref["iterates"][-1]
        Ug = mix[i][0].T
        assert ref["iters"] == mix[i][1]
        assert np.linalg.norm(Ug - Uo, axis=1).max() <= 1e-11 * np.linalg.norm(Uo, axis=1).max()


def test_serve_budget_admission(ctx, setup):
    P = setup[0]["P"]
    per_req = 2 * 8 * P.n * P.N
    reqs = [r for r in _requests() if r[0] == 0]
    free = _run(_server(ctx, setup), reqs, arrive_at=[0] * len(reqs))
    srv = _server(ctx, setup, budget=2 * per_req)
    ids = {}
    for i, (op, u0, f) in enumerate(reqs):
        rid, U = srv.submit(op, _dev(u0), _dev(f))
        ids[rid] = (i, U)
    got, peak = {}, 0
    while len(got) < len(reqs):
        fin = srv.progress(wait=True)
        st = srv.stats()
        peak = max(peak, st["active"])
        assert st["bytes_in_use"] <= 2 * per_req
        for rid, it in fin:
            i, U = ids[rid]
            got[i] = (U.cpu().numpy().copy(), it)
    srv.close()
    assert peak <= 2
    for i in range(len(reqs)):
        assert got[i][1] == free[i][1]
        assert np.array_equal(got[i][0], free[i][0])


def test_serve_equals_parareal_solve(ctx, setup):
    o = setup[0]
    P = o["P"]
    op, u0, f = _requests()[2]
    srv = _server(ctx, setup)
    served = _run(srv, [(op, u0, f)], arrive_at=[0])[0]
    srv.close()
    out = ctx.parareal_solve(o["coarse"], [o["F"]] * P.N, P.m, _dev(u0.reshape(-1, 1)), _dev(f.reshape(-1, 1)),
                             o["fsc"], tol=1e-12)
    assert out["iters"][0] == served[1]
    ref = out["U"][0].cpu().numpy()
    assert np.abs(served[0].T - ref).max() <= 1e-14 * np.abs(ref).max()
