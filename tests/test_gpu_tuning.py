"""GPU tests of the tunable launch shapes and the LU autotuner.

* the band LU does not depend on the number of workgroups per matrix: the
  FP64 factors of a batch of four operators (lrpr_factor_many) are the same
  bit for bit for every setting of LRPR_TUNE_LU_WGS, and equal the oracle's
  LU to rounding;
* lrpr_autotune_factor returns one of its candidates, stores it in the
  context, and factors made after it are unchanged;
* out-of-range settings are refused.
"""
import numpy as np
import pytest

from paper_2508_08873_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2508_08873_amd import lrpr
    c = lrpr.Context(0)
    yield c
    c.close()


def _ops():
    P = inputs.dar127s(N=2, m=2)
    return [o for s in (1, 2) for o in P.step_ops(s)]


def test_lu_independent_of_workgroups(ctx, ora):
    from paper_2508_08873_amd import lrpr
    ops = _ops()
    ref = None
    for wgs in (0, 17, 8, 5, 3, 1):
        ctx.tune_set(lrpr.TUNE_LU_WGS, wgs)
        assert ctx.tune_get(lrpr.TUNE_LU_WGS) == wgs
        facs = ctx.factor_many(ops, store_mask=lrpr.STORE_F64)
        lus = [F.lu_host() for F in facs]
        for F in facs:
            F.close()
        if ref is None:
            ref = lus
            o = ora.Operator(**{k: ops[2][k] for k in ("dim", "nx", "nu", "beta", "c", "dt")})
            assert np.abs(lus[2] - o.lu).max() <= 1e-12 * np.abs(o.lu).max()
        else:
            for a, b in zip(lus, ref):
                assert np.array_equal(a, b), "LU differs with %d workgroups per matrix" % wgs
    ctx.tune_set(lrpr.TUNE_LU_WGS, 0)


def test_autotune_factor(ctx):
    from paper_2508_08873_amd import lrpr
    P = inputs.tiny2d(nx=63)
    o = P.op_params()
    best, ms = ctx.autotune_factor(o["dim"], o["nx"], o["nu"], o["beta"], o["c"], o["dt"], count=24,
                                   store_mask=lrpr.STORE_F64)
    nb = (P.nx + 15) // 16
    assert 1 <= best <= nb + 9 and ms > 0
    assert ctx.tune_get(lrpr.TUNE_LU_WGS) == best
    with pytest.raises(lrpr.LrprError):
        ctx.tune_set(lrpr.TUNE_LU_WGS, 1000)
    with pytest.raises(lrpr.LrprError):
        ctx.tune_set(99, 1)
    ctx.tune_set(lrpr.TUNE_LU_WGS, 0)
