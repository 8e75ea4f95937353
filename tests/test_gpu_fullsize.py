"""GPU checks at the benchmark's full sizes, against the oracle on sampled
outputs it can compute one by one, or against properties that hold at any
size.

* 255^2 operator (n = 65025, b = 255): fine and adjoint sweeps of 16 columns,
  two columns recomputed by the oracle (per-column relative 1e-11 FP64,
  1e-5 FP32);
* 511^2 operator with the time-dependent diffusion of its first slice
  (n = 261121, b = 511): the same, FP64 and FP32;
* both operators through factors kept with spikes (partitioned fine sweeps);
* the timed configuration (255^2, FP32 fine solves and range finder, factors
  with the UL set so that substitutions run in pairs): one sweep of all 3200
  range-finder columns x 32 steps, forward and adjoint, on three sampled
  columns (1e-5); the FP32 rSVD build of 64 slices on the library's Philox
  Omega, one slice against the oracle's rSVD on the oracle's own draws
  (1e-5); the FP32-fine Parareal iterate a fixed point of the oracle's F_n
  on sampled slices;
* the full 255^2 pipeline in FP64 (64 slices, k = 40, p = 10, Parareal to
  1e-10) on the library's Philox Omega: two sampled slices' singular values
  and coarse products against the oracle's rSVD on its own draws of the
  same Omega (1e-11), and the Parareal iterates against the oracle's
  recursion run with the library's coarse factors (same iteration count,
  1e-11).
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


def _dev(a, dt=torch.float64):
    from paper_2508_08873_amd.lrpr import colmajor
    return colmajor(torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt))


_OPS = {}


def _oracle_op(ora, P, s=1):
    """Oracle operator (factorised) of slice s, shared by the tests of this module."""
    key = (P.name, s)
    if key not in _OPS:
        _OPS[key] = ora.Operator(**P.op_params(s))
    return _OPS[key]


def _sampled_sweep(ctx, ora, P, prec, adjoint, mirror, nsteps, cols=(3, 14), seed=5, split=False):
    from paper_2508_08873_amd import lrpr
    mask = (lrpr.STORE_F64 if prec == 0 else lrpr.STORE_F32 | lrpr.STORE_F64) | (lrpr.STORE_MIRROR if mirror else 0)
    mask |= lrpr.STORE_SPLIT if split else 0
    F = ctx.factor(P.dim, P.nx, P.nu_slice(1), P.beta, P.c, P.dt, store_mask=mask)
    X0 = np.random.default_rng(seed).standard_normal((P.n, 16))
    f = P.source()
    fsc = np.stack([P.fscale(1)[:nsteps]] * 16)
    dt = torch.float64 if prec == 0 else torch.float32
    X = _dev(X0, dt)
    spec = {"F": F, "X": X}
    if adjoint:
        ctx.adjoint_step_batched([spec], nsteps, prec)
    else:
        spec["f"] = _dev(f.reshape(-1, 1), dt)
        spec["fscale"] = torch.from_numpy(np.ascontiguousarray(fsc)).to("cuda")
        ctx.fine_step_batched([spec], nsteps, prec)
    got = X.double().cpu().numpy()
    F.close()
    op = _oracle_op(ora, P)
    Xs = X0[:, list(cols)]
    ref = op.adjoint(Xs, nsteps) if adjoint else op.fine(Xs, nsteps, f, None, fsc[: len(cols)])
    g = got[:, list(cols)]
    return float(np.max(np.linalg.norm(g - ref, axis=0) / np.linalg.norm(ref, axis=0)))


@pytest.mark.parametrize("adjoint,mirror", [(False, True), (True, True), (True, False)],
                         ids=["fwd", "adj_mirror", "adj_strided"])
def test_dar255_sweep_sampled(ctx, ora, adjoint, mirror):
    err = _sampled_sweep(ctx, ora, inputs.dar255(), 0, adjoint, mirror, nsteps=4)
    assert err <= 1e-11, err


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("adjoint", [False, True], ids=["fwd", "adj"])
def test_dar511t_sweep_sampled(ctx, ora, prec, adjoint):
    err = _sampled_sweep(ctx, ora, inputs.dar511t(), prec, adjoint, mirror=False, nsteps=2)
    assert err <= (1e-11 if prec == 0 else 1e-5), err


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("name", ["dar255", "dar511t"])
def test_partitioned_sweep_sampled(ctx, ora, name, prec):
    """Fine sweeps of one 16-column group through factors kept with spikes
    (partitioned passes; 16 and 32 band tiles)."""
    P = getattr(inputs, name)()
    print("case", name, "prec", prec, flush=True)
    err = _sampled_sweep(ctx, ora, P, prec, False, False, nsteps=2, split=True)
    assert err <= (1e-11 if prec == 0 else 1e-5), err


@pytest.fixture(scope="module")
def dar255_run(ctx):
    """The whole 255^2 pipeline in FP64 as the benchmark's FP64 side runs it
    (factor with the UL set, mirror and spikes; paired range-finder sweeps;
    partitioned Parareal sweeps), with Omega_n the library's Philox
    Gaussians of (seed 0, stream n), so that the oracle can redraw them."""
    from paper_2508_08873_amd import lrpr
    P = inputs.dar255()
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt,
                   store_mask=lrpr.STORE_F64 | lrpr.STORE_MIRROR | lrpr.STORE_SPLIT | lrpr.STORE_UL)
    Om = torch.empty((P.N, P.l, P.n), device="cuda", dtype=torch.float64)
    for s in range(P.N):
        ctx.randn(Om[s], 0, s)
    coarse = ctx.rsvd_build([(F, P.k, P.p, Om[s].t()) for s in range(P.N)], P.m, 0)
    del Om
    u0 = P.u0()
    f = P.source()
    fsc = torch.from_numpy(np.concatenate([P.fscale(s) for s in range(1, P.N + 1)])).to("cuda")
    out = ctx.parareal_solve(coarse, [F] * P.N, P.m, _dev(u0.reshape(-1, 1)), _dev(f.reshape(-1, 1)), fsc,
                             tol=P.tol)
    yield {"P": P, "F": F, "coarse": coarse, "out": out, "u0": u0, "f": f}
    coarse.close()
    F.close()


def _coarse_host(coarse, s, l):
    from paper_2508_08873_amd.lrpr import device_view
    k, n, U, S, V = coarse.get(s)
    return (device_view(U, n, k).cpu().numpy(), device_view(S, l, 1).cpu().numpy()[:, 0],
            device_view(V, n, k).cpu().numpy())


@pytest.mark.parametrize("s", [0, 40])
def test_dar255_rsvd_sampled_slices_f64(ctx, ora, dar255_run, s):
    """Sampled slices of the FP64 build against the oracle's randomized SVD
    (Sec. 2.1 steps 1-6) on the same Omega (the oracle's own Philox4x32-10 +
    Box-Muller draws): singular values (max |d sigma_j| / sigma_1) and the
    coarse product on a Gaussian probe within 1e-11."""
    from oracle import philox
    P, coarse = dar255_run["P"], dar255_run["coarse"]
    print("dar255 FP64 rsvd, slice", s + 1, flush=True)
    Om = philox.randn(P.l * P.n, 0, s).reshape(P.l, P.n).T
    Uo, So, Vo = ora.rsvd(_oracle_op(ora, P), P.m, P.k, P.p, Om)
    Ug, Sg, Vg = _coarse_host(coarse, s, P.l)
    assert np.array_equal(Sg, np.array(coarse.sigma[s * P.l:(s + 1) * P.l]))
    k = P.k
    X = np.random.default_rng(3).standard_normal((P.n, 16))
    Pg, Po = Ug @ (Sg[:k, None] * (Vg.T @ X)), Uo @ (So[:k, None] * (Vo.T @ X))
    es, ep = np.abs(Sg - So).max() / So[0], np.linalg.norm(Pg - Po) / np.linalg.norm(Po)
    print("dar255 FP64 rsvd: sigma error %.2e, product error %.2e, sigma_1 %.6f, sigma_k+1 %.3e"
          % (es, ep, So[0], So[k]), flush=True)
    assert es <= 1e-11 and ep <= 1e-11
    assert So[0] <= 1.0
    assert np.abs(Ug.T @ Ug - np.eye(k)).max() <= 1e-12
    assert np.abs(Vg.T @ Vg - np.eye(k)).max() <= 1e-12


def test_dar255_parareal_iterates_f64(ctx, ora, dar255_run):
    """The FP64 Parareal iterates against the oracle's Parareal recursion
    (eq. def_Parareal) run with the library's own coarse factors U_k, S_k,
    V_k (so the oracle computes the fine solves F_n, the b_n = F_n 0 and the
    correction itself): same iteration count, and the final iterate within
    1e-11 relative (max_n ||du_n|| / max_n ||u_n||)."""
    P, coarse, out = dar255_run["P"], dar255_run["coarse"], dar255_run["out"]
    assert out["status"] == 0
    op = _oracle_op(ora, P)
    sl = [ora.Slice(op, P.m, dar255_run["f"], P.fscale(n)) for n in range(1, P.N + 1)]
    for s in range(P.N):
        sl[s].Uk, sl[s].S, sl[s].Vk = _coarse_host(coarse, s, P.l)
    for s, b in zip(sl, ora.fine_all(sl, [np.zeros(P.n)] * P.N)):
        s.b = b
    print("dar255 FP64 parareal: oracle run with the library's coarse factors", flush=True)
    ref = ora.parareal(sl, dar255_run["u0"], tol=P.tol)
    Uo = ref["iterates"][-1]
    Ug = out["U"][0].cpu().numpy()
    err = np.linalg.norm(Ug - Uo, axis=1).max() / np.linalg.norm(Uo, axis=1).max()
    print("dar255 FP64 parareal: iterations %d (oracle %d), iterate error %.2e, increments %s"
          % (out["iters"][0], ref["iters"], err, ref["incr"]), flush=True)
    assert out["iters"][0] == ref["iters"]
    assert err <= 1e-11
    for k in range(ref["iters"]):
        assert abs(out["incr"][0][k] - ref["incr"][k]) <= 1e-11 * np.linalg.norm(Uo, axis=1).max()


# -- the timed configuration: FP32 fine solves and range finder on factors kept
# with the UL set (steps alternate L U / U' L', substitutions paired), 64 slices
# x (k + p) = 3200 range-finder columns x 32 steps in one sweep call

@pytest.fixture(scope="module")
def timed_factor(ctx):
    from paper_2508_08873_amd import lrpr
    P = inputs.dar255()
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt,
                   store_mask=lrpr.STORE_F64 | lrpr.STORE_F32 | lrpr.STORE_MIRROR | lrpr.STORE_SPLIT | lrpr.STORE_UL)
    yield P, F
    F.close()


@pytest.mark.parametrize("adjoint", [False, True], ids=["fwd", "adj"])
def test_timed_config_sweep_sampled(ctx, ora, timed_factor, adjoint):
    """One FP32 sweep of all 3200 columns over the 32 steps of a slice; three
    columns (first, inside, last group) from host draws, recomputed by the
    oracle; every other column is filled with torch Gaussians."""
    P, F = timed_factor
    w = P.N * P.l
    cols = (0, 1633, w - 1)
    print("timed config sweep, adjoint", adjoint, "w", w, flush=True)
    Xs = np.random.default_rng([21, int(adjoint)]).standard_normal((P.n, len(cols)))
    Xs = Xs.astype(np.float32).astype(np.float64)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(21)
    X = torch.randn((w, P.n), generator=gen, device="cuda", dtype=torch.float32).t()
    for j, c in enumerate(cols):
        X[:, c] = torch.from_numpy(Xs[:, j]).to("cuda", torch.float32)
    spec = {"F": F, "X": X}
    fsc = np.stack([P.fscale(1 + c // P.l) for c in range(w)])
    f = P.source()
    if adjoint:
        ctx.adjoint_step_batched([spec], P.m, 1)
    else:
        spec["f"] = _dev(f.reshape(-1, 1), torch.float32)
        spec["fscale"] = torch.from_numpy(np.ascontiguousarray(fsc)).to("cuda")
        ctx.fine_step_batched([spec], P.m, 1)
    got = X[:, list(cols)].double().cpu().numpy()
    op = _oracle_op(ora, P)
    ref = op.adjoint(Xs, P.m) if adjoint else op.fine(Xs, P.m, f, None, fsc[list(cols)])
    err = float(np.max(np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)))
    print("timed config sweep error", err, flush=True)
    assert err <= 1e-5, err


@pytest.fixture(scope="module")
def timed_run(ctx, timed_factor):
    """The FP32 rSVD build and Parareal (to 1e-6) of the timed step, with
    Omega_n the library's Philox Gaussians of (seed 0, stream n)."""
    P, F = timed_factor
    Om = torch.empty((P.N, P.l, P.n), device="cuda", dtype=torch.float64)
    for s in range(P.N):
        ctx.randn(Om[s], 0, s)
    Om32 = Om.to(torch.float32)
    del Om
    coarse = ctx.rsvd_build([(F, P.k, P.p, Om32[s].t()) for s in range(P.N)], P.m, 1)
    del Om32
    u0, f = P.u0(), P.source()
    fsc = torch.from_numpy(np.concatenate([P.fscale(s) for s in range(1, P.N + 1)])).to("cuda")
    out = ctx.parareal_solve(coarse, [F] * P.N, P.m, _dev(u0.reshape(-1, 1)), _dev(f.reshape(-1, 1)), fsc,
                             tol=1e-6, fine_prec=1)
    torch.cuda.synchronize()
    yield {"P": P, "coarse": coarse, "out": out, "u0": u0, "f": f}
    coarse.close()


def test_timed_config_rsvd_sampled_slice(ctx, ora, timed_run):
    """Slice 17 of the FP32 build against the oracle's randomized SVD on the
    same Omega (the oracle's own Philox4x32-10 + Box-Muller draws, rounded to
    FP32 as the library's range finder sees them): singular values and the
    coarse product on sampled vectors within 1e-5 (relative to sigma_1 and
    to the product's norm)."""
    from oracle import philox
    from paper_2508_08873_amd.lrpr import device_view
    P, coarse = timed_run["P"], timed_run["coarse"]
    s = 16
    print("timed config rsvd, slice", s + 1, flush=True)
    Om = philox.randn(P.l * P.n, 0, s).reshape(P.l, P.n).T.astype(np.float32).astype(np.float64)
    Uo, So, Vo = ora.rsvd(_oracle_op(ora, P), P.m, P.k, P.p, Om)
    Sg = np.array(coarse.sigma[s * P.l:(s + 1) * P.l])
    k, n, U, S, V = coarse.get(s)
    Ug, Vg = device_view(U, n, k).cpu().numpy(), device_view(V, n, k).cpu().numpy()
    Sk = device_view(S, P.l, 1).cpu().numpy()[:k, 0]
    X = np.random.default_rng(3).standard_normal((n, 4))
    Pg, Po = Ug @ (Sk[:, None] * (Vg.T @ X)), Uo @ (So[:k, None] * (Vo.T @ X))
    es, ep = np.abs(Sg - So).max() / So[0], np.linalg.norm(Pg - Po) / np.linalg.norm(Po)
    print("timed config rsvd: sigma error", es, "product error", ep, flush=True)
    assert es <= 1e-5, es
    assert ep <= 1e-5, ep
    # U_k = Q Uh and V_k = Q_Z Vh with Q, Q_Z orthonormalised from FP32 panels
    assert np.abs(Ug.T @ Ug - np.eye(k)).max() <= 1e-5
    assert np.abs(Vg.T @ Vg - np.eye(k)).max() <= 1e-5


def test_timed_config_parareal_fixed_point(ctx, ora, timed_run):
    """The FP32-fine Parareal iterate converged to 1e-6 satisfies
    u_n = F_n u_{n-1} on sampled slices to the FP32 fine solves' rounding
    (1e-5 of the largest state norm), F_n the oracle's FP64 propagator."""
    P, out = timed_run["P"], timed_run["out"]
    assert out["status"] == 0 and out["iters"][0] <= P.N
    U = out["U"][0].cpu().numpy()
    assert np.array_equal(U[0], timed_run["u0"])
    op = _oracle_op(ora, P)
    scale = np.linalg.norm(U, axis=1).max()
    for n_ in (1, 33, 64):
        ref = op.fine(U[n_ - 1].reshape(-1, 1), P.m, timed_run["f"], None, P.fscale(n_).reshape(1, -1))[:, 0]
        e = np.linalg.norm(U[n_] - ref) / scale
        print("timed config parareal: slice", n_, "fixed-point residual", e, flush=True)
        assert e <= 1e-5, n_


def test_fp32_smooth_mode_accuracy(ctx, ora):
    """FP32 tiles keep each row's sum when rounded, so 32 FP32 steps of the
    255^2 operator (L U factors, unpaired passes) shrink the smooth grid
    modes sin(pi x) sin(pi y) and sin(2 pi x) sin(pi y) by less than 1e-6
    forward and 3e-6 adjoint relative to the oracle (measured 3e-7 and
    2e-6; plainly rounded tiles gave 2.1e-6 and 3.9e-6).  The remaining
    error is the FP32 rounding of the partial sums, which is also nearly the
    same in every interior row; its size depends on how the kernel groups
    the band tiles, so a change of that grouping can move it within the
    FP32 target and needs these bounds re-measured."""
    from paper_2508_08873_amd import lrpr
    P = inputs.dar255()
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt,
                   store_mask=lrpr.STORE_F64 | lrpr.STORE_F32 | lrpr.STORE_MIRROR)
    x = np.arange(1, P.nx + 1) / (P.nx + 1)
    Xg, Yg = np.meshgrid(x, x, indexing="xy")
    V = np.stack([(np.sin(np.pi * Xg) * np.sin(np.pi * Yg)).reshape(-1),
                  (np.sin(2 * np.pi * Xg) * np.sin(np.pi * Yg)).reshape(-1)], axis=1)
    V = V.astype(np.float32).astype(np.float64)
    # padded to 16 columns so that the forward sweep runs on the matrix cores
    # (two columns alone take the vector-ALU sweep: test_fp32_smooth_mode_narrow)
    Vp = np.concatenate([V, np.random.default_rng(2).standard_normal((P.n, 14)).astype(np.float32)], axis=1)
    op = _oracle_op(ora, P)
    for adjoint in (False, True):
        print("smooth modes, adjoint", adjoint, flush=True)
        Xd = _dev(Vp, torch.float32)
        (ctx.adjoint_step_batched if adjoint else ctx.fine_step_batched)([{"F": F, "X": Xd}], P.m, 1)
        g = Xd.double().cpu().numpy()[:, :2]
        ref = op.adjoint(V, P.m) if adjoint else op.fine(V, P.m)
        err = np.linalg.norm(g - ref, axis=0) / np.linalg.norm(ref, axis=0)
        print("smooth-mode error", err, flush=True)
        assert err.max() <= (1e-6 if not adjoint else 3e-6), err
    F.close()


def test_fp32_smooth_mode_narrow(ctx, ora):
    """The same smooth modes through the vector-ALU sweep of narrow panels
    (two columns, FP32 products and sums): 32 steps of the 255^2 operator
    forward, against the oracle, within the FP32 target."""
    from paper_2508_08873_amd import lrpr
    P = inputs.dar255()
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt, store_mask=lrpr.STORE_F64 | lrpr.STORE_F32)
    x = np.arange(1, P.nx + 1) / (P.nx + 1)
    Xg, Yg = np.meshgrid(x, x, indexing="xy")
    V = np.stack([(np.sin(np.pi * Xg) * np.sin(np.pi * Yg)).reshape(-1),
                  (np.sin(2 * np.pi * Xg) * np.sin(np.pi * Yg)).reshape(-1)], axis=1)
    V = V.astype(np.float32).astype(np.float64)
    Xd = _dev(V, torch.float32)
    ctx.fine_step_batched([{"F": F, "X": Xd}], P.m, 1)
    g = Xd.double().cpu().numpy()
    ref = _oracle_op(ora, P).fine(V, P.m)
    err = np.linalg.norm(g - ref, axis=0) / np.linalg.norm(ref, axis=0)
    print("narrow smooth-mode error", err, flush=True)
    assert err.max() <= 5e-6, err
    F.close()


@pytest.mark.parametrize("nx,beta", [(255, (10.0, 5.0)), (127, (10.0, 5.0)), (127, (20.0, 10.0))],
                         ids=["255_b10", "127_b10", "127_b20"])
def test_fp32_accuracy_other_operators(ctx, ora, nx, beta):
    """32 FP32 steps, forward and adjoint, of two smooth grid modes and a
    random vector on further operators (nu = 1, c = 1, dt = 1/2048; 16 and 8
    band tiles), with paired U L / U' L' passes and with L U steps alone,
    against the oracle: measured at most 4.8e-7 paired and 1.1e-6 L U."""
    from paper_2508_08873_amd import lrpr
    dt = 1.0 / 2048
    op = ora.Operator(2, nx, 1.0, beta, 1.0, dt)
    x = np.arange(1, nx + 1) / (nx + 1)
    Xg, Yg = np.meshgrid(x, x, indexing="xy")
    V = np.stack([(np.sin(np.pi * Xg) * np.sin(np.pi * Yg)).reshape(-1),
                  (np.sin(2 * np.pi * Xg) * np.sin(np.pi * Yg)).reshape(-1),
                  np.random.default_rng(3).standard_normal(nx * nx)], axis=1)
    V = V.astype(np.float32).astype(np.float64)
    base = lrpr.STORE_F64 | lrpr.STORE_F32 | lrpr.STORE_MIRROR
    for ul, bound in ((True, 1e-6), (False, 2e-6)):
        F = ctx.factor(2, nx, 1.0, beta, 1.0, dt, store_mask=base | (lrpr.STORE_UL if ul else 0))
        for adjoint in (False, True):
            print("operator", nx, beta, "ul", ul, "adjoint", adjoint, flush=True)
            Xd = _dev(V, torch.float32)
            (ctx.adjoint_step_batched if adjoint else ctx.fine_step_batched)([{"F": F, "X": Xd}], 32, 1)
            g = Xd.double().cpu().numpy()
            ref = op.adjoint(V, 32) if adjoint else op.fine(V, 32)
            err = np.linalg.norm(g - ref, axis=0) / np.linalg.norm(ref, axis=0)
            assert err.max() <= bound, (ul, adjoint, err)
        F.close()
