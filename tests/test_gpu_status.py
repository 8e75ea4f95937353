"""GPU tests of the error statuses and of the Parareal outputs around them.

* a non-finite pivot in the band LU returns LRPR_ERR_ZERO_PIVOT;
* a non-finite initial value makes the Parareal increments non-finite:
  LRPR_ERR_NONFINITE;
* max_iter < N returns LRPR_ERR_NOCONV with every output written: the
  iterate after max_iter iterations equals the oracle's (1e-11), and the a
  posteriori bound (Thm. 3, eq. apost_bound) equals the oracle's bound
  evaluated on the library's own increments and singular values (1e-12);
* max_iter > N with several problems: the increments of problem r sit at
  incr + r * max_iter, the caller's stride, and equal each problem's own.
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
    a = np.ascontiguousarray(a)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    return colmajor(torch.from_numpy(a).to("cuda", torch.float64))


def _problem(ctx):
    from paper_2508_08873_amd import lrpr
    P = inputs.tiny2d(nx=21, N=6, m=4, k=5, p=3)
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt, store_mask=lrpr.STORE_F64 | lrpr.STORE_MIRROR)
    oms = [P.omega(s) for s in range(1, P.N + 1)]
    coarse = ctx.rsvd_build([(F, P.k, P.p, _dev(oms[s])) for s in range(P.N)], P.m, 0)
    fsc = torch.from_numpy(np.concatenate([P.fscale(s) for s in range(1, P.N + 1)])).to("cuda")
    return P, F, oms, coarse, fsc


@pytest.mark.parametrize("dim,nx", [(1, 8), (2, 20)])
def test_nonfinite_pivot(ctx, dim, nx):
    from paper_2508_08873_amd import lrpr
    # nu * dt / h^2 overflows: every pivot is infinite
    with pytest.raises(lrpr.LrprError) as ei:
        ctx.factor(dim, nx, 1e300, (0.0, 0.0), 0.0, 1e300, store_mask=lrpr.STORE_F64)
    assert ei.value.status == 3
    # the context stays usable
    F = ctx.factor(dim, nx, 1.0, (0.0, 0.0), 0.0, 1e-3, store_mask=lrpr.STORE_F64)
    F.close()


def test_nonfinite_increment(ctx):
    from paper_2508_08873_amd import lrpr
    P, F, oms, coarse, fsc = _problem(ctx)
    u0 = P.u0()
    u0[5] = np.nan
    with pytest.raises(lrpr.LrprError) as ei:
        ctx.parareal_solve(coarse, [F] * P.N, P.m, _dev(u0), _dev(P.source()), fsc, tol=1e-12)
    assert ei.value.status == 6
    # a finite problem on the same context still solves
    out = ctx.parareal_solve(coarse, [F] * P.N, P.m, _dev(P.u0()), _dev(P.source()), fsc, tol=1e-12)
    assert out["status"] == 0


def test_noconv_outputs_and_apost(ctx, ora):
    P, F, oms, coarse, fsc = _problem(ctx)
    u0, f = P.u0(), P.source()
    o1 = ctx.parareal_solve(coarse, [F] * P.N, P.m, _dev(u0), _dev(f), fsc, tol=0.0, max_iter=1)
    o2 = ctx.parareal_solve(coarse, [F] * P.N, P.m, _dev(u0), _dev(f), fsc, tol=0.0, max_iter=2)
    assert o1["status"] == 5 and o2["status"] == 5
    assert o1["iters"] == [1] and o2["iters"] == [2]
    U1 = o1["U"][0].cpu().numpy()
    U2 = o2["U"][0].cpu().numpy()
    # iterates against the oracle's Parareal (own rSVD of the same Omega)
    op = ora.Operator(**P.op_params())
    sl = [ora.Slice(op, P.m, f, P.fscale(s)) for s in range(1, P.N + 1)]
    ora.build_coarse(sl, P.k, P.p, oms)
    ref = ora.parareal(sl, u0, tol=0.0, max_iter=2)
    for k, Ug in ((1, U1), (2, U2)):
        Uo = ref["iterates"][k]
        err = np.linalg.norm(Ug - Uo, axis=1).max() / np.linalg.norm(Uo, axis=1).max()
        assert err <= 1e-11, (k, err)
        assert abs(ref["incr"][k - 1] - (o1 if k == 1 else o2)["incr"][0][k - 1]) <= 1e-11 * np.abs(Uo).max()
    # the increments of iteration 2 from the library's own iterates (the
    # max_iter = 2 run repeats iteration 1 bit for bit)
    inc = np.linalg.norm(U2[1:] - U1[1:], axis=1)
    assert abs(inc.max() - o2["incr"][0][1]) <= 1e-13 * inc.max()
    sig = np.array(coarse.sigma).reshape(P.N, P.l)
    delta, eps = sig[:, 0].max(), sig[:, P.k].max()
    want = ora.apost_bound(delta, eps, inc)
    got = np.array(o2["apost"][0])
    assert got[0] == 0.0
    assert np.abs(got - want).max() <= 1e-12 * want.max(), (got, want)
    # against the oracle's own constants and increments (iterates agree to 1e-11)
    do, eo = ora.bound_constants(sl, P.k)
    inc_o = np.linalg.norm(ref["iterates"][2][1:] - ref["iterates"][1][1:], axis=1)
    want_o = ora.apost_bound(do, eo, inc_o)
    assert np.abs(got - want_o).max() <= 1e-8 * want_o.max()


def test_max_iter_above_n_stride(ctx):
    P, F, oms, coarse, fsc = _problem(ctx)
    mi = P.N + 3
    u0 = np.stack([P.u0(req=r) for r in range(3)], axis=1)
    f = np.stack([P.source(req=r) for r in range(3)], axis=1)
    out = ctx.parareal_solve(coarse, [F] * P.N, P.m, _dev(u0), _dev(f), fsc, tol=1e-13, max_iter=mi)
    assert out["status"] == 0
    for r in range(3):
        one = ctx.parareal_solve(coarse, [F] * P.N, P.m, _dev(u0[:, r]), _dev(f[:, r]), fsc, tol=1e-13, max_iter=mi)
        K = one["iters"][0]
        assert out["iters"][r] == K and 1 <= K <= P.N
        row = out["incr"][r]
        assert len(row) == mi
        assert row[:K] == one["incr"][0][:K]
        assert all(v > 0 for v in row[:K]) and all(v == 0.0 for v in row[K:])
        assert np.array_equal(out["U"][r].cpu().numpy(), one["U"][0].cpu().numpy())
