"""GPU parity of the SDIRK fine steppers (lrpr_factor_stepper) against the
oracle's stage-by-stage implementation of the two tableaus (pinned to their
stability functions and to second-order convergence):

* forward sweeps with a source whose time factors differ per stage, and
  adjoint sweeps; plain and partitioned passes; FP64 (1e-11) and FP32 (1e-5);
* the rSVD of the SDIRK transfer operator and Parareal on SDIRK slices
  (FP64), against the oracle's rSVD and Parareal on the same stepper.
"""
import numpy as np
import pytest
import torch

from paper_2508_08873_amd import inputs

pytestmark = pytest.mark.gpu

METHODS = {"sdirk2": 1, "sdirk2l": 2}
TOL = {0: 1e-11, 1: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    from paper_2508_08873_amd import lrpr
    return lrpr.Context(0)


def _dev(a, dt=torch.float64):
    from paper_2508_08873_amd.lrpr import colmajor
    return colmajor(torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt))


def _colerr(got, ref):
    return float(np.max(np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)))


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("method", list(METHODS))
@pytest.mark.parametrize("nx,w,split", [(31, 21, False), (63, 9, True)], ids=["plain", "partitioned"])
def test_sdirk_sweeps(ctx, ora, method, prec, nx, w, split):
    from paper_2508_08873_amd import lrpr
    P = inputs.tiny2d(nx=nx, m=3)
    print("sdirk", method, "prec", prec, "nx", nx, "split", split, flush=True)
    pp = P.op_params()
    st = ora.Stepper(method, **pp)
    mask = lrpr.STORE_F64 | lrpr.STORE_F32 | (lrpr.STORE_SPLIT if split else lrpr.STORE_MIRROR)
    F = ctx.factor(pp["dim"], pp["nx"], pp["nu"], pp["beta"], pp["c"], pp["dt"], store_mask=mask,
                   stepper=METHODS[method])
    r = np.random.default_rng(17)
    X0 = r.standard_normal((P.n, w))
    f = P.source()
    fsc = 1.0 + 0.5 * r.standard_normal((w, 2 * P.m))   # stage time factors, two per step
    dt = torch.float64 if prec == 0 else torch.float32
    X = _dev(X0, dt)
    ctx.fine_step_batched([{"F": F, "X": X, "f": _dev(f.reshape(-1, 1), dt),
                            "fscale": torch.from_numpy(np.ascontiguousarray(fsc)).to("cuda")}], P.m, prec)
    torch.cuda.synchronize()
    ref = st.fine(X0, P.m, f, None, fsc)
    assert _colerr(X.double().cpu().numpy(), ref) <= TOL[prec]
    Y = _dev(X0, dt)
    ctx.adjoint_step_batched([{"F": F, "X": Y}], P.m, prec)
    torch.cuda.synchronize()
    assert _colerr(Y.double().cpu().numpy(), st.adjoint(X0, P.m)) <= TOL[prec]


@pytest.mark.parametrize("method", list(METHODS))
def test_sdirk_rsvd_and_parareal(ctx, ora, method):
    from paper_2508_08873_amd import lrpr
    P = inputs.tiny2d(nx=23, N=4, m=3, k=8, p=2, T=1.0 / 8)
    print("sdirk rsvd/parareal", method, flush=True)
    pp = P.op_params()
    st = ora.Stepper(method, **pp)
    F = ctx.factor(pp["dim"], pp["nx"], pp["nu"], pp["beta"], pp["c"], pp["dt"],
                   store_mask=lrpr.STORE_F64 | lrpr.STORE_MIRROR, stepper=METHODS[method])
    oms = [P.omega(s) for s in range(1, P.N + 1)]
    coarse = ctx.rsvd_build([(F, P.k, P.p, _dev(oms[s])) for s in range(P.N)], P.m, 0)
    l = P.k + P.p
    from paper_2508_08873_amd.lrpr import device_view
    for s in range(P.N):
        Uo, So, Vo = ora.rsvd_general(st, P.m, P.k, P.p, oms[s])
        Sg = np.array(coarse.sigma[s * l:(s + 1) * l])
        assert np.abs(Sg - So).max() <= 1e-11 * So[0], s
        k, n, U, S, V = coarse.get(s)
        Ug, Vg = device_view(U, n, k).cpu().numpy(), device_view(V, n, k).cpu().numpy()
        Sk = device_view(S, l, 1).cpu().numpy()[:k, 0]
        X = np.random.default_rng(7).standard_normal((n, 16))
        Pg, Po = Ug @ (Sk[:, None] * (Vg.T @ X)), Uo @ (So[:k, None] * (Vo.T @ X))
        assert np.linalg.norm(Pg - Po) <= 1e-11 * np.linalg.norm(Po), s
    # Parareal: source with stage time factors, same iteration count as the oracle
    cs = ora.TABLEAUS[method][0]
    f = P.source()
    u0 = P.u0()
    fsc = np.concatenate([P.fscale_stages(s, cs) * (1.0 + 0.1 * s) for s in range(1, P.N + 1)])
    out = ctx.parareal_solve(coarse, [F] * P.N, P.m, _dev(u0.reshape(-1, 1)), _dev(f.reshape(-1, 1)),
                             torch.from_numpy(fsc).to("cuda"), tol=P.tol)
    slices = [ora.Slice(st, P.m, f, fsc[(s - 1) * 2 * P.m:s * 2 * P.m].reshape(1, -1)) for s in range(1, P.N + 1)]
    ora.build_coarse(slices, P.k, P.p, oms)
    ref = ora.parareal(slices, u0, P.tol)
    assert out["status"] == 0
    assert out["iters"][0] == ref["iters"], (out["iters"][0], ref["iters"])
    Ug = out["U"][0].cpu().numpy()
    Uo = ref["iterates"][-1]
    scale = np.linalg.norm(Uo, axis=1).max()
    assert np.linalg.norm(Ug - Uo, axis=1).max() <= 1e-11 * scale
    seq = ora.sequential(slices, u0)
    assert np.linalg.norm(Ug - seq, axis=1).max() <= 1e-9 * scale
