"""GPU parity of per-step operators inside a slice (lrpr_factor_sequence:
one implicit-Euler factor per step, nu changing every step) against the
oracle's StepSequence: forward sweeps with a source and adjoint sweeps
(plain and partitioned, FP64 / FP32), and the rSVD and Parareal on slices
made of such sequences (FP64, the slices with different sequences)."""
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


def _dev(a, dt=torch.float64):
    from paper_2508_08873_amd.lrpr import colmajor
    return colmajor(torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt))


def _colerr(got, ref):
    return float(np.max(np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)))


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("nx,w,split", [(31, 19, False), (63, 7, True)], ids=["plain", "partitioned"])
def test_sequence_sweeps(ctx, ora, prec, nx, w, split):
    from paper_2508_08873_amd import lrpr
    P = inputs.tiny2d(nx=nx, m=4, nu_of_t=True, T=1.0 / 4)
    print("sequence prec", prec, "nx", nx, "split", split, flush=True)
    ops = P.step_ops(3)
    seq = ora.StepSequence(ops)
    mask = lrpr.STORE_F64 | lrpr.STORE_F32 | (lrpr.STORE_SPLIT if split else 0)
    F = ctx.factor_sequence(ops, store_mask=mask)
    r = np.random.default_rng(23)
    X0 = r.standard_normal((P.n, w))
    f = P.source()
    fsc = 1.0 + 0.3 * r.standard_normal((w, P.m))
    dt = torch.float64 if prec == 0 else torch.float32
    X = _dev(X0, dt)
    ctx.fine_step_batched([{"F": F, "X": X, "f": _dev(f.reshape(-1, 1), dt),
                            "fscale": torch.from_numpy(np.ascontiguousarray(fsc)).to("cuda")}], P.m, prec)
    torch.cuda.synchronize()
    assert _colerr(X.double().cpu().numpy(), seq.fine(X0, P.m, f, None, fsc)) <= TOL[prec]
    Y = _dev(X0, dt)
    ctx.adjoint_step_batched([{"F": F, "X": Y}], P.m, prec)
    torch.cuda.synchronize()
    assert _colerr(Y.double().cpu().numpy(), seq.adjoint(X0, P.m)) <= TOL[prec]
    # fewer steps than the sequence holds: the first steps (adjoint: their transposed product)
    Z = _dev(X0, dt)
    ctx.adjoint_step_batched([{"F": F, "X": Z}], 2, prec)
    torch.cuda.synchronize()
    assert _colerr(Z.double().cpu().numpy(), seq.adjoint(X0, 2)) <= TOL[prec]


def test_sequence_rsvd_and_parareal(ctx, ora):
    from paper_2508_08873_amd import lrpr
    P = inputs.tiny2d(nx=21, N=4, m=3, k=8, p=2, T=1.0 / 4, nu_of_t=True)
    facs, seqs = [], []
    for s in range(1, P.N + 1):
        ops = P.step_ops(s)
        seqs.append(ora.StepSequence(ops))
        facs.append(ctx.factor_sequence(ops, store_mask=lrpr.STORE_F64))
    oms = [P.omega(s) for s in range(1, P.N + 1)]
    coarse = ctx.rsvd_build([(facs[s], P.k, P.p, _dev(oms[s])) for s in range(P.N)], P.m, 0)
    l = P.k + P.p
    for s in range(P.N):
        Uo, So, Vo = ora.rsvd_general(seqs[s], P.m, P.k, P.p, oms[s])
        Sg = np.array(coarse.sigma[s * l:(s + 1) * l])
        assert np.abs(Sg - So).max() <= 1e-11 * So[0], s
    f, u0 = P.source(), P.u0()
    fsc = np.concatenate([P.fscale(s) for s in range(1, P.N + 1)])
    out = ctx.parareal_solve(coarse, facs, P.m, _dev(u0.reshape(-1, 1)), _dev(f.reshape(-1, 1)),
                             torch.from_numpy(fsc).to("cuda"), tol=P.tol)
    slices = [ora.Slice(seqs[s - 1], P.m, f, P.fscale(s).reshape(1, -1)) for s in range(1, P.N + 1)]
    ora.build_coarse(slices, P.k, P.p, oms)
    ref = ora.parareal(slices, u0, P.tol)
    assert out["status"] == 0 and out["iters"][0] == ref["iters"]
    Ug, Uo = out["U"][0].cpu().numpy(), ref["iterates"][-1]
    scale = np.linalg.norm(Uo, axis=1).max()
    assert np.linalg.norm(Ug - Uo, axis=1).max() <= 1e-11 * scale
    seq_ref = ora.sequential(slices, u0)
    assert np.linalg.norm(Ug - seq_ref, axis=1).max() <= 1e-9 * scale
