"""GPU parity of paired implicit-Euler sweeps (factors stored with
LRPR_STORE_UL: steps alternate between M = L U and M = U' L', and the last
substitution of one step shares its pass over the rows with the first of the
next) against the oracle's fine and adjoint propagators.

* forward sweeps with a source whose time factors differ per column and step,
  and adjoint sweeps; 8 and 16 band tiles per row (the paired kernels), odd
  and even step counts, a ragged last column group; FP64 (1e-11) and FP32
  (1e-5);
* the paired path really runs: for two or more steps its FP64 result differs
  in the last bits from the same sweep on a factor without the UL set (the
  other factorisation rounds differently) and agrees with it to 1e-12; for
  one step the two are the same launch and agree bit for bit;
* several panels with their own factors in one paired launch, and a launch
  that mixes band-tile counts (which falls back to unpaired passes);
* the rSVD build and Parareal on UL factors against the oracle.
"""
import numpy as np
import pytest
import torch

from paper_2508_08873_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {0: 1e-11, 1: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    from paper_2508_08873_amd import lrpr
    return lrpr.Context(0)


_OPS = {}


def _op(ora, P):
    key = (P.nx, P.nu, tuple(P.beta), P.c, P.dt)
    if key not in _OPS:
        _OPS[key] = ora.Operator(**P.op_params())
    return _OPS[key]


def _dev(a, prec=0):
    from paper_2508_08873_amd.lrpr import colmajor
    dt = torch.float64 if prec == 0 else torch.float32
    return colmajor(torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt))


def _colerr(got, ref):
    return float(np.max(np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)))


def _factor(ctx, P, ul=True, mirror=True):
    from paper_2508_08873_amd import lrpr
    mask = lrpr.STORE_F64 | lrpr.STORE_F32 | (lrpr.STORE_MIRROR if mirror else 0) | (lrpr.STORE_UL if ul else 0)
    return ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt, store_mask=mask)


def _sweep(ctx, F, P, X0, nsteps, prec, adjoint, fsc=None):
    X = _dev(X0, prec)
    spec = {"F": F, "X": X}
    if not adjoint and fsc is not None:
        spec["f"] = _dev(P.source().reshape(-1, 1), prec)
        spec["fscale"] = torch.from_numpy(np.ascontiguousarray(fsc)).to("cuda", torch.float64)
    if adjoint:
        ctx.adjoint_step_batched([spec], nsteps, prec)
    else:
        ctx.fine_step_batched([spec], nsteps, prec)
    torch.cuda.synchronize()
    return X.double().cpu().numpy()


# (name, problem, columns, steps): nx 121 has 8 band tiles per row, nx 250 has 16
CASES = [
    ("nb8_2steps", lambda: inputs.tiny2d(nx=121, m=3), 21, 2),
    ("nb8_3steps", lambda: inputs.tiny2d(nx=121, m=3, beta=(-12.0, 25.0)), 16, 3),
    ("nb16_2steps", lambda: inputs.tiny2d(nx=250, m=5, T=1.0 / 64), 17, 2),
    ("nb16_5steps", lambda: inputs.tiny2d(nx=250, m=5, T=1.0 / 64), 5, 5),
]


@pytest.mark.parametrize("name,mk,w,nsteps", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("adjoint", [False, True], ids=["fwd", "adj"])
def test_paired_sweep_parity(ctx, ora, name, mk, w, nsteps, prec, adjoint):
    P = mk()
    print("paired", name, "prec", prec, "adjoint", adjoint, flush=True)
    F = _factor(ctx, P)
    r = np.random.default_rng([5, w, nsteps])
    X0 = r.standard_normal((P.n, w))
    fsc = 1.0 + 0.5 * r.standard_normal((w, nsteps))   # own time factor per column and step
    op = _op(ora, P)
    ref = op.adjoint(X0, nsteps) if adjoint else op.fine(X0, nsteps, P.source(), None, fsc)
    got = _sweep(ctx, F, P, X0, nsteps, prec, adjoint, fsc)
    err = _colerr(got, ref)
    assert err <= TOL[prec], err
    F.close()


@pytest.mark.parametrize("adjoint", [False, True], ids=["fwd", "adj"])
def test_paired_path_runs(ctx, adjoint):
    P = inputs.tiny2d(nx=121, m=4)
    print("paired path check, adjoint", adjoint, flush=True)
    Fu = _factor(ctx, P, ul=True)
    Fp = _factor(ctx, P, ul=False)
    r = np.random.default_rng(11)
    X0 = r.standard_normal((P.n, 16))
    fsc = 1.0 + 0.1 * r.standard_normal((16, 4))
    for nsteps in (1, 2, 4):
        a = _sweep(ctx, Fu, P, X0, nsteps, 0, adjoint, fsc)
        b = _sweep(ctx, Fp, P, X0, nsteps, 0, adjoint, fsc)
        if nsteps == 1:
            assert np.array_equal(a, b)
        else:
            assert not np.array_equal(a, b), nsteps
            assert _colerr(a, b) <= 1e-12, (nsteps, _colerr(a, b))
    Fu.close()
    Fp.close()


def test_paired_multi_panel_and_mixed_fallback(ctx, ora):
    """Two factors with 8 band tiles per row in one paired launch (own
    sources and time factors); then a launch mixing 8 and 16 band tiles,
    which runs unpaired passes, on the same data."""
    P1 = inputs.tiny2d(nx=121, m=3)
    P2 = inputs.tiny2d(nx=127, m=3, beta=(20.0, -5.0))
    P3 = inputs.tiny2d(nx=250, m=3, T=1.0 / 64)
    nsteps = 3
    plans = [(P1, 21), (P2, 9)]
    for mixed in (False, True):
        if mixed:
            plans = plans + [(P3, 7)]
        print("paired multi-panel, mixed", mixed, flush=True)
        specs, refs, keep = [], [], []
        for i, (P, w) in enumerate(plans):
            F = _factor(ctx, P)
            r = np.random.default_rng([7, i])
            X0 = r.standard_normal((P.n, w))
            fsc = 1.0 + 0.3 * r.standard_normal((w, nsteps))
            specs.append({"F": F, "X": _dev(X0), "f": _dev(P.source().reshape(-1, 1)),
                          "fscale": torch.from_numpy(np.ascontiguousarray(fsc)).to("cuda")})
            refs.append(_op(ora, P).fine(X0, nsteps, P.source(), None, fsc))
            keep.append(F)
        ctx.fine_step_batched(specs, nsteps, 0)
        torch.cuda.synchronize()
        for sp, ref in zip(specs, refs):
            assert _colerr(sp["X"].cpu().numpy(), ref) <= 1e-11
        for F in keep:
            F.close()


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_paired_rsvd_and_parareal(ctx, ora, prec):
    """rSVD build (paired forward and adjoint range-finder sweeps) and
    Parareal on UL factors, against the oracle on the same Omega."""
    from paper_2508_08873_amd import lrpr
    from paper_2508_08873_amd.lrpr import device_view
    P = inputs.tiny2d(nx=121, N=4, m=4, k=12, p=4, T=1.0 / 8)
    print("paired rsvd/parareal prec", prec, flush=True)
    pp = P.op_params()
    F = ctx.factor(pp["dim"], pp["nx"], pp["nu"], pp["beta"], pp["c"], pp["dt"],
                   store_mask=lrpr.STORE_F64 | lrpr.STORE_F32 | lrpr.STORE_MIRROR | lrpr.STORE_UL)
    oms = [P.omega(s) for s in range(1, P.N + 1)]
    coarse = ctx.rsvd_build([(F, P.k, P.p, _dev(oms[s], prec)) for s in range(P.N)], P.m, prec)
    l = P.k + P.p
    op = _op(ora, P)
    tol = TOL[prec]
    for s in range(P.N):
        Uo, So, Vo = ora.rsvd(op, P.m, P.k, P.p, oms[s])
        Sg = np.array(coarse.sigma[s * l:(s + 1) * l])
        assert np.abs(Sg - So).max() <= tol * So[0], (s, np.abs(Sg - So).max() / So[0])
        k, n, U, S, V = coarse.get(s)
        Ug, Vg = device_view(U, n, k).cpu().numpy(), device_view(V, n, k).cpu().numpy()
        Sk = device_view(S, l, 1).cpu().numpy()[:k, 0]
        X = np.random.default_rng(3).standard_normal((n, 8))
        Pg, Po = Ug @ (Sk[:, None] * (Vg.T @ X)), Uo @ (So[:k, None] * (Vo.T @ X))
        assert np.linalg.norm(Pg - Po) <= tol * np.linalg.norm(Po), s
    if prec == 0:
        f = P.source()
        u0 = P.u0()
        fsc = np.concatenate([P.fscale(s) for s in range(1, P.N + 1)])
        out = ctx.parareal_solve(coarse, [F] * P.N, P.m, _dev(u0.reshape(-1, 1)), _dev(f.reshape(-1, 1)),
                                 torch.from_numpy(fsc).to("cuda"), tol=P.tol)
        slices = [ora.Slice(op, P.m, f, P.fscale(s)) for s in range(1, P.N + 1)]
        ora.build_coarse(slices, P.k, P.p, oms)
        ref = ora.parareal(slices, u0, P.tol)
        assert out["status"] == 0
        assert out["iters"][0] == ref["iters"], (out["iters"][0], ref["iters"])
        Ug = out["U"][0].cpu().numpy()
        Uo = ref["iterates"][-1]
        scale = np.linalg.norm(Uo, axis=1).max()
        assert np.linalg.norm(Ug - Uo, axis=1).max() <= 1e-11 * scale
    coarse.close()
    F.close()
