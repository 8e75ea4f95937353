"""GPU parity on the uneven batch: problems of the 48-problem draw (grid 63^2 to
255^2, rank k ~ U{8..64}, p = floor(k/4), own nu, beta, c) go through ONE
randomized-SVD build and ONE batched fine sweep, each slice with its own
factor, size and rank.

* 63^2 and 127^2 slices: singular values and coarse products against the
  oracle's rSVD on the same Omega (FP64 1e-11, FP32 range finder 1e-5);
* the 255^2 slice: orthonormal U_k, V_k, descending sigma with sigma_1 <= 1,
  and the low-rank error on a sampled vector within a few sigma_{k+1} of the
  oracle's T v (eq. truncation_error);
* the mixed fine sweep: every column against the oracle's fine propagator.
"""
import numpy as np
import pytest
import torch

from paper_2508_08873_amd import inputs

pytestmark = pytest.mark.gpu

# (problem index in the draw, slice): two slices of problem 1 share its factor
PICKS = [(1, 1), (1, 2), (4, 1), (6, 1), (7, 1), (14, 1)]
FULL_CHECK_NX = (63, 127)


@pytest.fixture(scope="module")
def ctx():
    from paper_2508_08873_amd import lrpr
    return lrpr.Context(0)


@pytest.fixture(scope="module")
def problems():
    return inputs.uneven48()


_OPS = {}


def _op(ora, P):
    if P.name not in _OPS:
        _OPS[P.name] = ora.Operator(**P.op_params(1))
    return _OPS[P.name]


def _dev(a, dtype=torch.float64):
    from paper_2508_08873_amd.lrpr import colmajor
    return colmajor(torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype))


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_uneven_rsvd_batch(ctx, ora, problems, prec):
    from paper_2508_08873_amd import lrpr
    from paper_2508_08873_amd.lrpr import device_view
    dt = torch.float64 if prec == 0 else torch.float32
    facs = {}
    entries, oms = [], []
    for i, s in PICKS:
        P = problems[i]
        if i not in facs:
            pp = P.op_params(s)
            facs[i] = ctx.factor(pp["dim"], pp["nx"], pp["nu"], pp["beta"], pp["c"], pp["dt"],
                                 store_mask=lrpr.STORE_F64 | lrpr.STORE_F32 | lrpr.STORE_MIRROR)
        om = P.omega(s)
        oms.append(om)
        entries.append((facs[i], P.k, P.p, _dev(om, dt)))
    print("uneven rsvd batch", [(problems[i].nx, problems[i].k, problems[i].p) for i, _ in PICKS], "prec", prec,
          flush=True)
    coarse = ctx.rsvd_build(entries, 32, prec)
    torch.cuda.synchronize()
    tol = 1e-11 if prec == 0 else 1e-5
    off = 0
    for e, (i, s) in enumerate(PICKS):
        P = problems[i]
        l = P.k + P.p
        Sg = np.array(coarse.sigma[off:off + l])
        off += l
        k, n, U, S, V = coarse.get(e)
        assert (k, n) == (P.k, P.n)
        Ug = device_view(U, n, k).cpu().numpy()
        Vg = device_view(V, n, k).cpu().numpy()
        Sk = device_view(S, l, 1).cpu().numpy()[:k, 0]
        assert np.all(np.diff(Sg) <= 1e-15 * Sg[0])
        assert Sg[0] <= 1.0 + 1e-12
        if P.nx in FULL_CHECK_NX:
            Uo, So, Vo = ora.rsvd(_op(ora, P), P.m, P.k, P.p, oms[e])
            assert np.abs(Sg - So).max() <= tol * So[0], (i, np.abs(Sg - So).max() / So[0])
            X = np.random.default_rng(7).standard_normal((n, 16))
            Pg = Ug @ (Sk[:, None] * (Vg.T @ X))
            Po = Uo @ (So[:k, None] * (Vo.T @ X))
            assert np.linalg.norm(Pg - Po) / np.linalg.norm(Po) <= tol, i
        else:
            I = np.eye(k)
            assert np.abs(Ug.T @ Ug - I).max() <= 1e-12 * (1 if prec == 0 else 1e6)
            assert np.abs(Vg.T @ Vg - I).max() <= 1e-12 * (1 if prec == 0 else 1e6)
            v = np.random.default_rng(9).standard_normal((n, 1))
            Tv = _op(ora, P).fine(v, P.m)
            err = np.linalg.norm(Tv - Ug @ (Sk[:, None] * (Vg.T @ v))) / np.linalg.norm(v)
            assert err <= 10.0 * Sg[k] + (1e-13 if prec == 0 else 1e-5), (i, err, Sg[k])
    coarse.close()
    for F in facs.values():
        F.close()


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_uneven_fine_sweep_mixed(ctx, ora, problems, prec):
    """One batched fine sweep over panels of three sizes (63^2, 127^2, 255^2),
    each with its own factor, source and per-column time factors."""
    from paper_2508_08873_amd import lrpr
    dt = torch.float64 if prec == 0 else torch.float32
    nsteps = 8
    plan = [(1, 5), (7, 20), (14, 3)]
    specs, refs, keep = [], [], []
    for i, w in plan:
        P = problems[i]
        pp = P.op_params(1)
        F = ctx.factor(pp["dim"], pp["nx"], pp["nu"], pp["beta"], pp["c"], pp["dt"],
                       store_mask=lrpr.STORE_F64 | lrpr.STORE_F32)
        X0 = np.random.default_rng([3, i]).standard_normal((P.n, w))
        f = P.source()
        fsc = np.stack([P.fscale(1 + (c % P.N))[:nsteps] for c in range(w)])
        X = _dev(X0, dt)
        specs.append({"F": F, "X": X, "f": _dev(f.reshape(-1, 1), dt),
                      "fscale": torch.from_numpy(np.ascontiguousarray(fsc)).to("cuda")})
        refs.append(_op(ora, P).fine(X0, nsteps, f, None, fsc))
        keep.append(F)
    print("uneven mixed sweep prec", prec, flush=True)
    ctx.fine_step_batched(specs, nsteps, prec)
    torch.cuda.synchronize()
    for sp, ref in zip(specs, refs):
        got = sp["X"].double().cpu().numpy()
        err = np.max(np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0))
        assert err <= (1e-11 if prec == 0 else 1e-5), err
    for F in keep:
        F.close()
