"""FP32 sweeps that carry several 16-column groups per workgroup (one band
tile load feeding the products of up to three groups).

Each group keeps the one-group sweep's order of operations, so the results
must equal the one-group sweep's bit for bit; against the oracle the FP32
bound of the other sweep tests (1e-5 per column) applies.
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
    c.tune_set(lrpr.TUNE_SWEEP_GROUPS, 0)


def _dev(a, dtype=torch.float32):
    from paper_2508_08873_amd.lrpr import colmajor
    return colmajor(torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype))


def _specs(P, F, X0, with_src, nsteps):
    X = _dev(X0)
    spec = {"F": F, "X": X}
    if with_src:
        w = X0.shape[1]
        f = np.stack([P.source(), 0.5 * P.source()[::-1].copy()], axis=1)
        spec["f"] = _dev(f)
        spec["fcol"] = torch.tensor([c % 3 - 1 for c in range(w)], dtype=torch.int32, device="cuda")
        fsc = np.stack([P.fscale(1 + (c % P.N)) for c in range(w)])[:, :nsteps]
        spec["fscale"] = torch.from_numpy(np.ascontiguousarray(fsc)).to("cuda", torch.float64)
    return spec


def _sweep(ctx, specs, nsteps, adjoint, groups):
    from paper_2508_08873_amd import lrpr
    ctx.tune_set(lrpr.TUNE_SWEEP_GROUPS, groups)
    (ctx.adjoint_step_batched if adjoint else ctx.fine_step_batched)(specs, nsteps, lrpr.LRPR_F32)
    torch.cuda.synchronize()


# band classes 8 (nx = 100), 16 (nx = 255) and 32 (nx = 300: 19 band tiles)
GRIDS = [(100, 2), (255, 2), (300, 1)]


@pytest.mark.parametrize("nx,m", GRIDS, ids=["nx100", "nx255", "nx300"])
@pytest.mark.parametrize("mode", ["fine_src", "adjoint_mirror", "adjoint_strided"])
def test_groups_equal_one_group_bitwise(ctx, nx, m, mode):
    from paper_2508_08873_amd import lrpr
    P = inputs.tiny2d(nx=nx, m=m)
    adjoint = mode != "fine_src"
    mask = lrpr.STORE_F32 | (lrpr.STORE_MIRROR if mode == "adjoint_mirror" else 0)
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt, store_mask=mask)
    for w in (41, 80):
        X0 = np.random.default_rng([nx, w]).standard_normal((P.n, w))
        outs = []
        for groups in (1, 2, 3):
            print("nx", nx, "mode", mode, "w", w, "groups", groups, flush=True)
            spec = _specs(P, F, X0, not adjoint, m)
            _sweep(ctx, [spec], m, adjoint, groups)
            outs.append(spec["X"].clone())
        assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    F.close()


@pytest.mark.parametrize("mode", ["fine_src", "adjoint_strided"])
def test_groups_parity(ctx, ora, mode):
    """Three groups per workgroup (41 columns: 16 + 16 + 9) against the oracle."""
    from paper_2508_08873_amd import lrpr
    P = inputs.tiny2d(nx=255, m=2)
    nsteps, w = 2, 41
    adjoint = mode != "fine_src"
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt, store_mask=lrpr.STORE_F32)
    op = ora.Operator(**P.op_params())
    X0 = np.random.default_rng(7).standard_normal((P.n, w))
    spec = _specs(P, F, X0, not adjoint, nsteps)
    if adjoint:
        ref = op.adjoint(X0, nsteps)
    else:
        f = spec["f"].double().cpu().numpy()
        fcol = spec["fcol"].cpu().numpy()
        fsc = spec["fscale"].cpu().numpy()
        ref = np.empty_like(X0)
        # the oracle takes one source column per call: group the columns by it
        for fc in (-1, 0, 1):
            cols = np.nonzero(fcol == fc)[0]
            src = f[:, fc] if fc >= 0 else None
            ref[:, cols] = op.fine(X0[:, cols], nsteps, src, None, fsc[cols] if src is not None else None)
    _sweep(ctx, [spec], nsteps, adjoint, 3)
    got = spec["X"].double().cpu().numpy()
    err = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
    print("max column error", err.max(), flush=True)
    assert err.max() <= 1e-5, err
    F.close()


def test_groups_multi_panel_and_default(ctx):
    """Panels of different factors and widths in one launch (groups merge
    within a panel only), and the default group count on a launch with more
    than one workgroup per compute unit, against the one-group sweep."""
    from paper_2508_08873_amd import lrpr
    Pa, Pb = inputs.tiny2d(nx=100, m=2), inputs.tiny2d(nx=120, m=2, beta=(-6.0, 14.0))
    Fa = ctx.factor(Pa.dim, Pa.nx, Pa.nu, Pa.beta, Pa.c, Pa.dt, store_mask=lrpr.STORE_F32)
    Fb = ctx.factor(Pb.dim, Pb.nx, Pb.nu, Pb.beta, Pb.c, Pb.dt, store_mask=lrpr.STORE_F32)
    r = np.random.default_rng(11)
    layout = [(Pa, Fa, 20), (Pb, Fb, 48), (Pa, Fa, 5), (Pb, Fb, 33)]
    X0s = [r.standard_normal((P.n, w)) for P, F, w in layout]

    def run(groups, reps=1):
        specs = [_specs(P, F, X0, True, 2) for (P, F, w), X0 in zip(layout * reps, X0s * reps)]
        _sweep(ctx, specs, 2, False, groups)
        return [s["X"] for s in specs]

    one, three = run(1), run(3)
    for a, b in zip(one, three):
        assert torch.equal(a, b)
    # 96 copies of the layout: 864 groups in 384 items of up to three
    print("default group count, 384 panels", flush=True)
    many = run(0, reps=96)
    for i, x in enumerate(many):
        assert torch.equal(x, one[i % 4])
    Fa.close()
    Fb.close()


def test_groups_tune_range(ctx):
    from paper_2508_08873_amd import lrpr
    for v in (0, 1, 2, 3):
        ctx.tune_set(lrpr.TUNE_SWEEP_GROUPS, v)
        assert ctx.tune_get(lrpr.TUNE_SWEEP_GROUPS) == v
    with pytest.raises(lrpr.LrprError):
        ctx.tune_set(lrpr.TUNE_SWEEP_GROUPS, 4)
    ctx.tune_set(lrpr.TUNE_SWEEP_GROUPS, 0)


@pytest.mark.parametrize("prec,groups", [(0, 1), (1, 1), (1, 3)], ids=["f64", "f32", "f32_groups3"])
def test_mixed_band_classes_parity(ctx, ora, prec, groups):
    """One launch over factors of 2, 4, 16 and 17 band tiles per row (the
    launch runs the widest class's kernel; the narrower factors' surplus
    bulk tiles must read zero tiles against ring slots of their own)."""
    from paper_2508_08873_amd import lrpr
    probs = [inputs.tiny2d(nx=31, m=2), inputs.tiny2d(nx=63, m=2, beta=(-4.0, 9.0)),
             inputs.tiny2d(nx=255, m=2), inputs.tiny2d(nx=260, m=2, beta=(12.0, 3.0))]
    widths = [19, 35, 16, 33]
    dt = torch.float64 if prec == 0 else torch.float32
    specs, refs, facs = [], [], []
    for i, (P, w) in enumerate(zip(probs, widths)):
        F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt, store_mask=lrpr.STORE_F64 | lrpr.STORE_F32)
        facs.append(F)
        X0 = np.random.default_rng(40 + i).standard_normal((P.n, w))
        refs.append(ora.Operator(**P.op_params()).fine(X0, 2))
        specs.append({"F": F, "X": _dev(X0, dt)})
    ctx.tune_set(lrpr.TUNE_SWEEP_GROUPS, groups)
    ctx.fine_step_batched(specs, 2, prec)
    torch.cuda.synchronize()
    ctx.tune_set(lrpr.TUNE_SWEEP_GROUPS, 0)
    tol = 1e-11 if prec == 0 else 1e-5
    for sp, ref, P in zip(specs, refs, probs):
        got = sp["X"].double().cpu().numpy()
        err = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
        print("nx", P.nx, "max column error", err.max(), flush=True)
        assert np.isfinite(err).all() and err.max() <= tol, (P.nx, err.max())
    for F in facs:
        F.close()
