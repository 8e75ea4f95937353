"""Benchmark of the low-rank Parareal hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec f32|f64]

One step is one pass of the whole hot path over the 255x255
diffusion-advection-reaction workload (n = 65025 unknowns, half-bandwidth
255, nu = 1, beta = (20, 10), c = 1, T = 1, 64 slices x 32 implicit-Euler
steps, rank k = 40, oversampling p = 10):
  1. assemble M = I + dt A and factor it (band LU, FP64) and pack the tiles;
  2. rSVD build of all 64 slices' transfer operators (3200 forward + 3200
     adjoint right-hand sides x 32 steps, CholeskyQR2, Jacobi SVD, rotation);
  3. Parareal to max_n ||u^{k+1}_n - u^k_n|| < tol (b_n sweep, coarse
     initialisation, iterations of 64 batched fine solves + sequential
     low-rank correction).
Precision: the fine solves and the range finder run in FP32 by default (FP32
accumulation; tol 1e-6), with the LU, the CholeskyQR2 Gram and Cholesky, the
Jacobi SVD and the Parareal correction and residual in FP64; --prec f64 runs
everything in FP64 (tol 1e-10).  The f32 run also times the FP64 form once
("fp64_side") and states the FP32 error against the FP64 oracle.
Inputs (Omega, u0, f) are generated before the timed region and stay in HBM.
`value` = fine-propagator RHS*steps per second of whole-step wall time, with
the K timed steps spread over --pipelines independent pipelines (default 3:
three library contexts, each on its own HIP stream, driven by its own host
thread), so that one step's LU, Parareal chain and small kernels fill the
compute units another's range-finder sweep leaves free (2 pipelines: 282 ms
per step, 3: 259 ms, 4: 286 ms on the 255^2 workload).  Each step is still
the whole path for one problem; the per-step latency of one pipeline alone,
its phase times and the sweep roofline come from a separate single-pipeline
timed run of K steps ("latency").

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import threading
import time

import numpy as np

PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
# Parareal tolerance of the FP32 configuration: FP32 fine solves move the
# fixed point by ~1e-6 relative, so it iterates to 1e-6 (FP64: 1e-10)
TOL_F32 = 1e-6
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["dar511t", "dar255", "uneven48", "serve3"], default="dar511t",
                    help="timed workload: the 511^2 time-dependent one (default; the 255^2 results ride along "
                         "as a side field), the 255^2 one alone, the 48 uneven problems, or serving at load")
    ap.add_argument("--no-side", action="store_true", help="dar511t: skip the 255^2 side run")
    ap.add_argument("--c1-steps", type=int, default=6, help="timed steps of the 255^2 side run")
    ap.add_argument("--fp64-steps", type=int, default=5, help="timed steps of the 255^2 FP64 side run")
    ap.add_argument("--c2-cpu-cols", type=int, default=64, help="oracle sample width on the 511^2 operator")
    ap.add_argument("--pipelines", type=int, default=3,
                    help="independent pipelines (context + stream + host thread) sharing the timed steps")
    ap.add_argument("--prec", choices=["f64", "f32"], default="f32",
                    help="fine solves and range finder (LU, Gram/Cholesky, SVD and the Parareal correction are "
                         "FP64 either way)")
    ap.add_argument("--no-fp64-side", action="store_true", help="skip the FP64 side run of the f32 bench")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-cols", type=int, default=384)
    ap.add_argument("--cpu-steps", type=int, default=32)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-RHS FP64 run")
    ap.add_argument("--no-ul", action="store_true",
                    help="factor without the UL set (every step L U, unpaired substitution passes)")
    ap.add_argument("--serve-rate", type=float, default=None,
                    help="Poisson arrival rate (requests/s; default 4 in the 255^2 run's serving study, 200 for "
                         "--workload serve3)")
    ap.add_argument("--serve-duration", type=float, default=None,
                    help="arrival window (s; default 15 in the serving study, 60 for --workload serve3)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (calibrates the HBM byte counters)")
    return ap.parse_args()


def copy_calib(mib):
    """Plain copy kernel of known size: reading FETCH_SIZE / WRITE_SIZE for it
    gives the factor between the counters and the bytes actually moved."""
    import torch
    nel = mib * (1 << 20) // 8
    src = torch.ones(nel, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calib_bytes_read": nel * 8, "copy_calib_bytes_written": nel * 8, "launches": 5}))


def cpu_baseline_and_parity(ctx, lrpr, P, prec, ncols, nsteps, seed):
    """Oracle fine propagator on a bounded sample of the workload (ncols
    right-hand sides x nsteps steps of the 255^2 operator, with the source
    term), timed on the host cores; the same sample runs through the GPU
    path and the per-column relative error is reported."""
    import torch
    import oracle
    oracle.build(force=False)
    op = oracle.Operator(**P.op_params())
    r = np.random.default_rng([seed, 99])
    X0 = r.standard_normal((P.n, ncols))
    f = P.source()
    fsc = np.stack([P.fscale(1 + (c % P.N))[:nsteps] for c in range(ncols)])
    threads = min(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), (ncols + 7) // 8)
    t0 = time.perf_counter()
    ref = op.fine(X0, nsteps, f, None, fsc)
    t1 = time.perf_counter()
    dt = torch.float64 if prec == "f64" else torch.float32
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt,
                   store_mask=(1 if prec == "f64" else 3) | lrpr.STORE_MIRROR | lrpr.STORE_SPLIT | UL_MASK[0])
    X = lrpr.colmajor(torch.from_numpy(X0).to("cuda", dt))
    spec = {"F": F, "X": X, "f": lrpr.colmajor(torch.from_numpy(f.reshape(-1, 1)).to("cuda", dt)),
            "fscale": torch.from_numpy(np.ascontiguousarray(fsc)).to("cuda")}
    ctx.fine_step_batched([spec], nsteps, 0 if prec == "f64" else 1)
    torch.cuda.synchronize()
    got = X.double().cpu().numpy()
    err = float(np.max(np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)))
    F.close()
    rate = ncols * nsteps / (t1 - t0)
    return {"value": rate, "unit": "RHS*steps/s", "cores": threads, "kind": "oracle",
            "sample": "%d RHS x %d implicit-Euler steps of the 255^2 operator with source (FP64 C oracle, "
                      "OpenMP over RHS columns), %.1f s" % (ncols, nsteps, t1 - t0)}, err


def serve_bench(ctx, lrpr, inputs, seed, rate, duration):
    """Serving workload: three operators (127^2, 255^2, 511^2; nu=1,
    beta=(10,5), c=1, 64 slices x 32 steps, k=48, p=12) with device-resident
    coarse propagators; requests (new u0 and f each, operator uniform) arrive
    as a Poisson stream and are served by lrpr_server with continuous batching,
    FP64 fine steps, tolerance 1e-8.  Latency = completion - arrival."""
    import torch
    probs = inputs.serve3(seed=seed)
    ops = []
    t_setup = time.perf_counter()
    for P in probs:
        F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt,
                       store_mask=lrpr.STORE_F64 | lrpr.STORE_MIRROR | lrpr.STORE_SPLIT)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed * 1000 + P.nx)
        Om = torch.randn((P.N, P.l, P.n), generator=gen, device="cuda", dtype=torch.float64)
        coarse = ctx.rsvd_build([(F, P.k, P.p, Om[s].t()) for s in range(P.N)], P.m, 0)
        del Om
        fsc = torch.from_numpy(np.concatenate([P.fscale(s) for s in range(1, P.N + 1)])).to("cuda")
        ops.append((coarse, [F] * P.N, P.m, fsc))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    arr = inputs.arrivals(seed=seed, rate=rate, duration=duration)
    r = inputs.rng(seed, "request", 0)
    which = r.integers(0, len(probs), size=len(arr))
    reqs = []
    for i, op in enumerate(which):
        P = probs[op]
        reqs.append((int(op), lrpr.colmajor(torch.from_numpy(P.u0(req=i + 1)).to("cuda").reshape(-1, 1)),
                     lrpr.colmajor(torch.from_numpy(P.source(req=i + 1)).to("cuda").reshape(-1, 1))))
    torch.cuda.synchronize()
    srv = lrpr.Server(ctx, ops, tol=probs[0].tol, budget_bytes=64 << 30)
    arrival, opof, lat, iters = {}, {}, {}, {}
    nxt = 0
    t0 = time.perf_counter()
    while len(lat) < len(reqs):
        now = time.perf_counter() - t0
        while nxt < len(reqs) and arr[nxt] <= now:
            op, u0, f = reqs[nxt]
            rid, _ = srv.submit(op, u0, f, sync=False)
            arrival[rid], opof[rid] = arr[nxt], op
            nxt += 1
        fin = srv.progress(wait=False)
        tnow = time.perf_counter() - t0
        for rid, it in fin:
            lat[rid] = tnow - arrival[rid]
            iters[rid] = it
        if not fin:
            time.sleep(0.0005)
    t_end = time.perf_counter() - t0
    srv.close()
    L = np.array([lat[k] for k in sorted(lat)])
    per_op = {}
    for o, P in enumerate(probs):
        lo = np.array([lat[k] for k in lat if opof[k] == o])
        if len(lo):
            per_op[P.name] = {"requests": int(len(lo)), "p50_s": float(np.percentile(lo, 50)),
                              "p99_s": float(np.percentile(lo, 99)),
                              "mean_iters": float(np.mean([iters[k] for k in iters if opof[k] == o]))}
    for c in ops:
        c[0].close()
        c[1][0].close()
    return {"workload": "serve3: operators 127^2, 255^2, 511^2 (nu=1, beta=(10,5), c=1, 64 slices x 32 steps, "
                        "k=48, p=12), Poisson arrivals %.1f/s for %.0f s, new u0 (8x8 sine modes) and f (1-6 "
                        "bumps) per request, FP64 fine steps, tol 1e-8" % (rate, duration),
            "requests": int(len(L)), "p50_s": float(np.percentile(L, 50)), "p99_s": float(np.percentile(L, 99)),
            "solves_per_s": float(len(L) / t_end), "wall_s": t_end, "setup_s": t_setup,
            "failed": int(sum(1 for v in iters.values() if v < 0)), "per_operator": per_op}


def c4_bench(ctx, lrpr, inputs, args):
    """Serving at the specified load: three operators (127^2, 255^2, 511^2;
    nu=1, beta=(10,5), c=1, 64 slices x 32 steps, k=48, p=12) with
    device-resident coarse propagators (FP64 rSVD, Philox Omega), Poisson
    arrivals at --serve-rate (default here 200/s) for --serve-duration
    (60 s), operator uniform, FP64 fine steps, tolerance 1e-8.  Requests wait
    in the client's FIFO and are handed to lrpr_server while its queue holds
    fewer than 64; latency = completion - arrival (queueing included).  After
    the arrivals stop, the run drains for at most 60 s; requests still open
    then are reported as unfinished (their latency exceeds the run).  The
    measured capacity (completions per second while the server was never
    idle) sets a second run at 0.7 x capacity, drained to the end.  Each
    request's u0 and f are drawn per request index modulo 32 (per operator)
    from the serving distribution (8x8 sine modes, 1-6 bumps).  The plain
    per-request FP64 path for comparison: the sequential fine solution of one
    request (64 x 32 implicit-Euler steps, one right-hand side, FP64
    partitioned passes), per operator."""
    import collections
    import torch
    probs = inputs.serve3(seed=args.seed)
    ops, pools = [], []
    t_setup = time.perf_counter()
    for oi, P in enumerate(probs):
        F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt,
                       store_mask=lrpr.STORE_F64 | lrpr.STORE_MIRROR | lrpr.STORE_SPLIT)
        Om = torch.empty((P.N, P.l, P.n), device="cuda", dtype=torch.float64)
        for s_ in range(P.N):
            ctx.randn(Om[s_], args.seed, 50000 + 1000 * oi + s_)
        coarse = ctx.rsvd_build([(F, P.k, P.p, Om[s_].t()) for s_ in range(P.N)], P.m, 0)
        del Om
        fsc = torch.from_numpy(np.concatenate([P.fscale(s_) for s_ in range(1, P.N + 1)])).to("cuda")
        ops.append((coarse, [F] * P.N, P.m, fsc))
        pools.append([(lrpr.colmajor(torch.from_numpy(P.u0(req=j + 1)).to("cuda").reshape(-1, 1)),
                       lrpr.colmajor(torch.from_numpy(P.source(req=j + 1)).to("cuda").reshape(-1, 1)))
                      for j in range(32)])
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    print("serve3: setup %.1f s" % t_setup, file=sys.stderr, flush=True)

    def run(rate, duration, drain, tag):
        arr = inputs.arrivals(seed=args.seed, rate=rate, duration=duration)
        which = inputs.rng(args.seed, "request", 0).integers(0, len(probs), size=len(arr))
        srv = lrpr.Server(ctx, ops, tol=probs[0].tol, budget_bytes=64 << 30)
        waiting = collections.deque()
        arrival, opof, lat, iters = {}, {}, {}, {}
        nxt, busy_t, last_report = 0, 0.0, 0.0
        t0 = time.perf_counter()
        while True:
            now = time.perf_counter() - t0
            while nxt < len(arr) and arr[nxt] <= now:
                waiting.append(nxt)
                nxt += 1
            st = srv.stats()
            while waiting and st["queued"] < 64:
                i = waiting.popleft()
                op = int(which[i])
                u0, f = pools[op][i % 32]
                rid, _ = srv.submit(op, u0, f, sync=False)
                arrival[rid], opof[rid] = arr[i], op
                st["queued"] += 1
            fin = srv.progress(wait=False)
            tnow = time.perf_counter() - t0
            for rid, it in fin:
                lat[rid] = tnow - arrival[rid]
                iters[rid] = it
            if st["active"] > 0 or st["queued"] > 0:
                busy_t = tnow
            if tnow - last_report > 10.0:
                print("serve3 %s: t=%.0f s, arrived %d, done %d, client queue %d" % (tag, tnow, nxt, len(lat),
                                                                                    len(waiting)),
                      file=sys.stderr, flush=True)
                last_report = tnow
            if nxt == len(arr) and not waiting and len(lat) == len(arrival):
                break
            if tnow > duration + drain:
                break
            if not fin:
                time.sleep(0.0005)
        wall = time.perf_counter() - t0
        srv.close()
        done = np.array([lat[k] for k in sorted(lat)]) if lat else np.zeros(1)
        per_op = {}
        for o, P in enumerate(probs):
            lo = np.array([lat[k] for k in lat if opof[k] == o])
            if len(lo):
                per_op[P.name] = {"done": int(len(lo)), "p50_s": float(np.percentile(lo, 50)),
                                  "p99_s": float(np.percentile(lo, 99))}
        return {"rate_per_s": rate, "arrival_s": duration, "arrived": int(len(arr)), "done": int(len(lat)),
                "unfinished": int(len(arr) - len(lat)), "wall_s": wall,
                "solves_per_s": float(len(lat) / max(busy_t, 1e-9)),
                "p50_s": float(np.percentile(done, 50)), "p99_s": float(np.percentile(done, 99)),
                "failed": int(sum(1 for v in iters.values() if v < 0)), "per_operator": per_op}

    rate = args.serve_rate if args.serve_rate is not None else 200.0
    duration = args.serve_duration if args.serve_duration is not None else 60.0
    sat = run(rate, duration, 60.0, "saturation")
    cap = sat["solves_per_s"]
    sus = run(0.7 * cap, duration, 120.0, "0.7 x capacity")
    # plain per-request FP64: the sequential fine solution of one request
    plain = {}
    for oi, P in enumerate(probs):
        coarse, facs, m, fsc = ops[oi]
        u0, f = pools[oi][0]
        X = lrpr.colmajor(u0.clone())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s_ in range(P.N):
            ctx.fine_step_batched([{"F": facs[0], "X": X, "f": f,
                                    "fscale": fsc[s_ * m:(s_ + 1) * m].reshape(1, -1).contiguous()}], m, 0)
        torch.cuda.synchronize()
        plain[P.name] = time.perf_counter() - t0
    plain_rate = 1.0 / float(np.mean(list(plain.values())))
    for c in ops:
        c[0].close()
        c[1][0].close()
    return {"workload": "serve3: operators 127^2, 255^2, 511^2 (nu=1, beta=(10,5), c=1, 64 slices x 32 steps, "
                        "k=48, p=12), Poisson arrivals, operator uniform, FP64 fine steps, tol 1e-8",
            "setup_s": t_setup, "saturation": sat, "capacity_solves_per_s": cap, "sustained": sus,
            "plain_per_request_fp64_s": plain, "plain_per_request_solves_per_s": plain_rate,
            "served_vs_plain_solves": cap / plain_rate}


def plain_per_rhs(ctx, lrpr, P, reps=8):
    """Plain per-RHS FP64 form: one right-hand side through the fine
    propagator (m steps, with source) per call, on the library's best
    single-RHS path (a factor with spikes: the partitioned passes spread the
    column over P compute units), timed with the library's events over
    `reps` calls.  The HBM fraction uses the algorithmic bytes of one RHS
    step (2 n s of state and n (2b+1) s of factor, s = 8)."""
    import torch
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt, store_mask=lrpr.STORE_F64 | lrpr.STORE_SPLIT)
    X = lrpr.colmajor(torch.zeros((P.n, 1), dtype=torch.float64, device="cuda"))
    f = lrpr.colmajor(torch.from_numpy(P.source().reshape(-1, 1)).to("cuda"))
    fsc = torch.from_numpy(P.fscale(1).reshape(1, -1).copy()).to("cuda")
    spec = {"F": F, "X": X, "f": f, "fscale": fsc}
    ctx.fine_step_batched([spec], P.m, 0)
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(reps):
        ctx.fine_step_batched([spec], P.m, 0)
    p = ctx.profile_read()
    ctx.profile(False)
    F.close()
    rate = reps * P.m / (p["ms"] / 1000.0)
    gbs = p["bytes"] / (p["ms"] / 1000.0) / 1e9
    return {"rhs_steps_per_s": rate, "path": "partitioned passes (factor with spikes), FP64",
            "algorithmic_GBs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS, "ms_per_call": p["ms"] / reps}


def fwd_adj_rates(ctx, lrpr, P, prec):
    """Forward and adjoint band sweeps reported separately: the range finder's
    width (N*l = 3200 RHS of the shared factor, m steps, no source), one
    launch each, timed with the library's events."""
    import torch
    fp = 0 if prec == "f64" else 1
    dt = torch.float64 if prec == "f64" else torch.float32
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt,
                   store_mask=(1 if prec == "f64" else 3) | lrpr.STORE_MIRROR | UL_MASK[0])
    gen = torch.Generator(device="cuda")
    gen.manual_seed(12345)
    X = torch.randn((P.N * P.l, P.n), generator=gen, device="cuda", dtype=dt).t()
    out = {}
    for name, call in (("forward", ctx.fine_step_batched), ("adjoint", ctx.adjoint_step_batched)):
        ctx.profile(True)
        call([{"F": F, "X": X}], P.m, fp)
        p = ctx.profile_read()
        ctx.profile(False)
        out[name + "_rhs_steps_per_s"] = p["rhs_steps"] / (p["ms"] / 1000.0)
        out[name + "_ms"] = p["ms"]
    out["rhs"] = P.N * P.l
    F.close()
    return out


def neumann_study(ctx, lrpr, seed):
    """The Neumann variant of the paper's first experiment (Sec. 4): 1D heat
    equation with homogeneous Neumann boundaries (255 points, nu = 1, 16
    slices x 32 implicit-Euler steps on [0, 4]: every non-constant mode
    decays by at least exp(-pi^2/4) per slice), whose constant mode is not
    damped.  Parareal to 1e-8 (at most N iterations) with four coarse
    solvers G_n = G_n' + b_n: G_n' = 0; the a priori rank-1 constant mode
    (U = 1, S = 1, V = W 1, L^2 inner product of the lumped mass W); the
    rank-8 randomized generalized SVD in that inner product; and the rank-8
    Euclidean rSVD."""
    import torch
    nx, N, m, T = 255, 16, 32, 4.0
    dt = T / (N * m)
    F = ctx.factor(1, nx, 1.0, (0.0, 0.0), 0.0, dt, store_mask=lrpr.STORE_F64 | lrpr.STORE_MIRROR | lrpr.STORE_SPLIT,
                   bc=lrpr.BC_NEUMANN)
    x = np.linspace(0.0, 1.0, nx)
    r = np.random.default_rng([seed, 255])
    u0 = 1.0 + np.cos(np.pi * x) + 0.5 * np.cos(4 * np.pi * x) + 0.05 * r.standard_normal(nx)
    f = np.exp(-40.0 * (x - 0.3) ** 2)
    fsc = np.cos(0.5 * np.pi * dt * np.arange(1, N * m + 1))
    dev = lambda a: lrpr.colmajor(torch.from_numpy(np.ascontiguousarray(a).reshape(nx, -1)).to("cuda"))
    w = lrpr.mass_weights(1, nx, lrpr.BC_NEUMANN)
    wd = torch.from_numpy(w).to("cuda")
    k, p = 8, 4
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed * 7 + 1)
    Om = torch.randn((N, k + p, nx), generator=gen, device="cuda", dtype=torch.float64)
    one = torch.ones(1, dtype=torch.float64, device="cuda")
    coarse = {
        "zero": ctx.coarse_from_factors([F] * N, [dev(np.zeros(nx))] * N, [0 * one] * N, [dev(np.zeros(nx))] * N),
        "constant_mode_rank1": ctx.coarse_from_factors([F] * N, [dev(np.ones(nx))] * N, [one] * N, [dev(w)] * N),
        "rsvd_L2_rank8": ctx.rsvd_build([(F, k, p, Om[s].t()) for s in range(N)], m, 0, weights=[wd] * N),
        "rsvd_euclidean_rank8": ctx.rsvd_build([(F, k, p, Om[s].t()) for s in range(N)], m, 0),
    }
    out = {"workload": "heat1d Neumann: 255 points, nu=1, 16 slices x 32 steps, T=4, tol 1e-8"}
    for name, C in coarse.items():
        t0 = time.perf_counter()
        o = ctx.parareal_solve(C, [F] * N, m, dev(u0), dev(f), torch.from_numpy(fsc).to("cuda"), tol=1e-8,
                               max_iter=N)
        torch.cuda.synchronize()
        out[name] = {"iters": o["iters"][0], "converged": o["status"] == 0, "s": time.perf_counter() - t0}
        C.close()
    F.close()
    return out


def rsvd_variants(ctx, lrpr, P, prec, Om):
    """rSVD build of the 64 slices, timed once each: the one-sided build
    (q = 0), with q = 1 power iteration (2 more sweeps of the 3200-column
    panel), and the two-sided build (adjoint on independent test vectors
    Psi); eps = max_n sigma_{n,k+1} of each."""
    import torch
    fp = 0 if prec == "f64" else 1
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt,
                   store_mask=(1 if prec == "f64" else 3) | lrpr.STORE_MIRROR | UL_MASK[0])
    Psi = torch.empty(Om.shape, device="cuda", dtype=torch.float64)
    for s_ in range(P.N):
        ctx.randn(Psi[s_], 777, s_)
    Psi = Psi.to(Om.dtype)
    out = {}
    for name, kw in (("q0", {}), ("q1", {"q": 1}), ("two_sided", {"psi": [Psi[s].t() for s in range(P.N)]})):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        coarse = ctx.rsvd_build([(F, P.k, P.p, Om[s].t()) for s in range(P.N)], P.m, fp, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sig = np.array(coarse.sigma).reshape(P.N, P.l)
        out[name] = {"rsvd_s": dt, "eps_max_sigma_k1": float(sig[:, P.k].max())}
        coarse.close()
    F.close()
    return out


def stepper_study(ctx, lrpr, P, prec, Om):
    """The paper's study of the time discretisation on this workload:
    implicit Euler, SDIRK2 and SDIRK2-L as fine steppers (same Omega): rSVD
    build time, eps = max_n sigma_{n,k+1} and sigma_{n,1} of the transfer
    operators, Parareal iterations and time to the bench tolerance."""
    import torch
    fp = 0 if prec == "f64" else 1
    tol = P.tol if prec == "f64" else TOL_F32
    u0 = lrpr.colmajor(torch.from_numpy(P.u0().reshape(-1, 1)).to("cuda"))
    f = lrpr.colmajor(torch.from_numpy(P.source().reshape(-1, 1)).to("cuda"))
    cs = {lrpr.STEP_SDIRK2: (1.0, 0.0), lrpr.STEP_SDIRK2L: ((2 - math.sqrt(2)) / 2, 1.0)}
    out = {}
    for name, stp in (("euler", lrpr.STEP_EULER), ("sdirk2", lrpr.STEP_SDIRK2), ("sdirk2l", lrpr.STEP_SDIRK2L)):
        F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt,
                       store_mask=(1 if prec == "f64" else 3) | lrpr.STORE_MIRROR | lrpr.STORE_SPLIT, stepper=stp)
        if stp == lrpr.STEP_EULER:
            fsc = np.concatenate([P.fscale(s) for s in range(1, P.N + 1)])
        else:
            fsc = np.concatenate([P.fscale_stages(s, cs[stp]) for s in range(1, P.N + 1)])
        fsc = torch.from_numpy(fsc).to("cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        coarse = ctx.rsvd_build([(F, P.k, P.p, Om[s].t()) for s in range(P.N)], P.m, fp)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = ctx.parareal_solve(coarse, [F] * P.N, P.m, u0, f, fsc, tol=tol, fine_prec=fp)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        sig = np.array(coarse.sigma).reshape(P.N, P.l)
        out[name] = {"rsvd_s": t1 - t0, "parareal_s": t2 - t1, "parareal_iters": int(res["iters"][0]),
                     "eps_max_sigma_k1": float(sig[:, P.k].max()), "delta_max_sigma_1": float(sig[:, 0].max())}
        coarse.close()
        F.close()
    return out


def per_step_operators(ctx, lrpr, inputs, prec, seed):
    """Per-step operators inside a slice (time-dependent coefficients): the
    127^2 workload with nu changing every step, 16 slices x 8 steps = 128
    band LUs, then the rSVD (k = 20, p = 5) and Parareal.  Reports the factor,
    rSVD and Parareal times: here the band LU is the dominant cost."""
    import torch
    P = inputs.dar127s(seed=seed)
    fp = 0 if prec == "f64" else 1
    tol = P.tol if prec == "f64" else TOL_F32
    mask = (1 if prec == "f64" else 3) | lrpr.STORE_MIRROR | lrpr.STORE_SPLIT
    Om = torch.empty((P.N, P.l, P.n), device="cuda", dtype=torch.float64)
    for s_ in range(P.N):
        ctx.randn(Om[s_], seed + 1, s_)
    Om = Om if prec == "f64" else Om.to(torch.float32)
    u0 = lrpr.colmajor(torch.from_numpy(P.u0().reshape(-1, 1)).to("cuda"))
    f = lrpr.colmajor(torch.from_numpy(P.source().reshape(-1, 1)).to("cuda"))
    fsc = torch.from_numpy(np.concatenate([P.fscale(s) for s in range(1, P.N + 1)])).to("cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    facs = [ctx.factor_sequence(P.step_ops(s), store_mask=mask) for s in range(1, P.N + 1)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    coarse = ctx.rsvd_build([(facs[s], P.k, P.p, Om[s].t()) for s in range(P.N)], P.m, fp)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out = ctx.parareal_solve(coarse, facs, P.m, u0, f, fsc, tol=tol, fine_prec=fp)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    sig = np.array(coarse.sigma).reshape(P.N, P.l)
    coarse.close()
    for F in facs:
        F.close()
    return {"workload": "dar127s: 127^2 grid, nu(t) per implicit-Euler step, 16 slices x 8 steps (128 band LUs), "
                        "k=20, p=5, Parareal to %g" % tol,
            "factors": P.N * P.m, "factor_s": t1 - t0, "rsvd_s": t2 - t1, "parareal_s": t3 - t2,
            "parareal_iters": int(out["iters"][0]), "eps_max_sigma_k1": float(sig[:, P.k].max())}


def c2_problem(seed):
    from paper_2508_08873_amd import inputs
    return inputs.dar511t(seed=seed)


def c2_bench(ctx, lrpr, args):
    """The 511^2 workload with time-dependent coefficients: nu_n = 1 + 0.5
    sin(2 pi t_n) per slice (128 slices x 16 implicit-Euler steps, dt =
    1/2048), so each slice has its own operator and band LU; k = 64, p = 16.
    One step:
      1. assemble and factor the 128 operators (band LU in FP64, tiles stored
         in FP32: 146 GB);
      2. rSVD build of all 128 slices together (128 x 80 = 10240 forward and
         10240 adjoint right-hand sides x 16 steps in FP32, one sweep launch
         each way; CholeskyQR2 Gram and Cholesky, Jacobi SVD and rotations in
         FP64), its panels in the workspace the LU bands used;
      3. Parareal with FP32 fine solves (one right-hand side per slice and
         factor, the HBM-bound regime) and the FP64 correction to
         max_n ||u^{k+1}_n - u^k_n|| < 1e-6, with the per-slice a posteriori
         bound (Thm. 3) from the computed singular values.
    Inputs (Omega in FP32 from the library's Philox generator, u0, f) are in
    HBM before the timed region.  Returns the result dict and the profile
    records."""
    import torch
    P = c2_problem(args.seed)
    ops = [P.op_params(s) for s in range(1, P.N + 1)]
    torch.cuda.empty_cache()
    Om = torch.empty((P.N, P.l, P.n), device="cuda", dtype=torch.float32)
    for s_ in range(P.N):
        ctx.randn(Om[s_], args.seed, s_)
    u0 = lrpr.colmajor(torch.from_numpy(P.u0().reshape(-1, 1)).to("cuda"))
    f = lrpr.colmajor(torch.from_numpy(P.source().reshape(-1, 1)).to("cuda"))
    fsc = torch.from_numpy(np.concatenate([P.fscale(s) for s in range(1, P.N + 1)])).to("cuda")
    torch.cuda.synchronize()
    # the library's autotuner picks the band LU's workgroups per matrix for
    # this batch (before the timed region; it does not change the factors)
    o1 = ops[0]
    tune = ctx.autotune_factor(o1["dim"], o1["nx"], o1["nu"], o1["beta"], o1["c"], o1["dt"], P.N,
                               store_mask=lrpr.STORE_F32)
    ctx.release_workspaces()

    def one_step(recs, times):
        ta = time.perf_counter()
        facs = ctx.factor_many(ops, store_mask=lrpr.STORE_F32)
        tb = time.perf_counter()
        coarse = ctx.rsvd_build([(facs[s], P.k, P.p, Om[s].t()) for s in range(P.N)], P.m, 1)
        tc = time.perf_counter()
        if recs is not None:
            recs["range"].append(ctx.profile_read())
        out = ctx.parareal_solve(coarse, facs, P.m, u0, f, fsc, tol=TOL_F32, fine_prec=1)
        torch.cuda.synchronize()
        td = time.perf_counter()
        if recs is not None:
            recs["parareal"].append(ctx.profile_read())
        sig = np.array(coarse.sigma).reshape(P.N, P.l)
        if times is not None:
            times.append((tb - ta, tc - tb, td - tc))
        coarse.close()
        for F in facs:
            F.close()
        return out, sig

    for _ in range(args.warmup):
        one_step(None, None)
    torch.cuda.synchronize()
    ctx.profile(True)
    recs = {"range": [], "parareal": []}
    times = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out, sig = one_step(recs, times)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile(False)
    del Om
    torch.cuda.empty_cache()
    ctx.device_trim()   # the pool's free blocks back to the device for what follows
    return P, out, sig, recs, times, t1 - t0, tune


def c2_cpu_baseline(P, ncols, nsteps, seed):
    """Oracle fine propagator on a bounded sample of the 511^2 workload:
    ncols right-hand sides x nsteps implicit-Euler steps (with the source)
    of slice 1's operator, timed on the host cores after the oracle's band
    LU of that operator (timed separately)."""
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    op = oracle.Operator(**P.op_params(1))
    t1 = time.perf_counter()
    r = np.random.default_rng([seed, 511])
    X0 = r.standard_normal((P.n, ncols))
    fsc = np.tile(P.fscale(1)[:nsteps], (ncols, 1))
    threads = min(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), ncols)
    t2 = time.perf_counter()
    op.fine(X0, nsteps, P.source(), None, fsc)
    t3 = time.perf_counter()
    return {"value": ncols * nsteps / (t3 - t2), "unit": "RHS*steps/s", "cores": threads, "kind": "oracle",
            "sample": "%d RHS x %d implicit-Euler steps of slice 1's 511^2 operator with source (FP64 C oracle, "
                      "OpenMP over RHS columns), %.1f s; the oracle's band LU of that operator took %.1f s "
                      "(not in the rate)" % (ncols, nsteps, t3 - t2, t1 - t0)}


def c3_bench(ctx, lrpr, inputs, args):
    """48 independent problems of uneven grid (63^2..511^2), operator, rank
    (k = 8..64, p = k/4) and slice count (N = 16, 32, 64), 32 implicit-Euler
    steps per slice, T = 1.  One pass:
      1. the band LUs, batched per grid (FP64 LU; FP32 and FP64 tiles);
      2. ONE rSVD build over all 1856 slices of the 48 problems (FP32 range
         finder: every slice's forward and adjoint right-hand sides in one
         sweep launch each way);
      3. ONE batched Parareal over the 48 problems (FP64 fine solves, tol
         1e-8 per problem; each problem stops on its own), each on a view of
         its slices' coarse propagators.
    Error per problem: the converged iterate against the sequential FP64
    fine solution u_n = F_n(u_{n-1}) computed afterwards on the GPU.
    Returns the result dict."""
    import torch
    probs = inputs.uneven48(seed=args.seed)
    tol = 1e-8
    # inputs in HBM: Omega per slice (library Philox, FP32), u0, f, time factors
    Oms, u0s, fs, fscs = [], [], [], []
    for i, P in enumerate(probs):
        Om = torch.empty((P.N, P.l, P.n), device="cuda", dtype=torch.float32)
        for s_ in range(P.N):
            ctx.randn(Om[s_], args.seed, 1000 * (i + 1) + s_)
        Oms.append(Om)
        u0s.append(lrpr.colmajor(torch.from_numpy(P.u0().reshape(-1, 1)).to("cuda")))
        fs.append(lrpr.colmajor(torch.from_numpy(P.source().reshape(-1, 1)).to("cuda")))
        fscs.append(torch.from_numpy(np.concatenate([P.fscale(n) for n in range(1, P.N + 1)])).to("cuda"))
    torch.cuda.synchronize()
    grids = sorted(set(P.nx for P in probs))
    t0 = time.perf_counter()
    facs = [None] * len(probs)
    for nx in grids:
        idx = [i for i, P in enumerate(probs) if P.nx == nx]
        got = ctx.factor_many([probs[i].op_params(1) for i in idx], store_mask=lrpr.STORE_F64 | lrpr.STORE_F32)
        for i, F in zip(idx, got):
            facs[i] = F
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print("uneven48: %d factors in %.2f s" % (len(facs), t1 - t0), file=sys.stderr, flush=True)
    slices, first = [], []
    for i, P in enumerate(probs):
        first.append(len(slices))
        slices += [(facs[i], P.k, P.p, Oms[i][s_].t()) for s_ in range(P.N)]
    ctx.profile(True)
    coarse = ctx.rsvd_build(slices, 32, 1)
    rng = ctx.profile_read()
    t2 = time.perf_counter()
    print("uneven48: rSVD build of %d slices in %.2f s" % (len(slices), t2 - t1), file=sys.stderr, flush=True)
    probs_in = [{"coarse": coarse.view(first[i], P.N), "factors": [facs[i]] * P.N, "u0": u0s[i], "f": fs[i],
                 "fscale": fscs[i], "tol": tol} for i, P in enumerate(probs)]
    outs = ctx.parareal_solve_many(probs_in, 32, fine_prec=0)
    torch.cuda.synchronize()
    par = ctx.profile_read()
    ctx.profile(False)
    t3 = time.perf_counter()
    print("uneven48: Parareal of %d problems in %.2f s" % (len(probs), t3 - t2), file=sys.stderr, flush=True)
    # sequential FP64 fine solution, slice index by slice index over all problems
    seq = [torch.zeros((P.N + 1, P.n), dtype=torch.float64, device="cuda") for P in probs]
    for i in range(len(probs)):
        seq[i][0] = u0s[i][:, 0]
    for s_ in range(max(P.N for P in probs)):
        specs = []
        for i, P in enumerate(probs):
            if s_ < P.N:
                X = lrpr.colmajor(seq[i][s_].clone().reshape(-1, 1))
                specs.append((i, {"F": facs[i], "X": X, "f": fs[i],
                                  "fscale": fscs[i][s_ * P.m:(s_ + 1) * P.m].reshape(1, -1).contiguous()}))
        ctx.fine_step_batched([sp for _, sp in specs], 32, 0)
        for i, sp in specs:
            seq[i][s_ + 1] = sp["X"][:, 0]
    torch.cuda.synchronize()
    errs, iters, per_grid = [], [], {}
    for i, P in enumerate(probs):
        U = outs[i]["U"][0]
        e = float((U - seq[i]).norm(dim=1).max() / seq[i].norm(dim=1).max())
        errs.append(e)
        iters.append(outs[i]["iters"][0])
        g = per_grid.setdefault("%d^2" % P.nx, {"problems": 0, "max_err": 0.0, "iters": []})
        g["problems"] += 1
        g["max_err"] = max(g["max_err"], e)
        g["iters"].append(outs[i]["iters"][0])
    for pr in probs_in:
        pr["coarse"].close()
    coarse.close()
    for F in facs:
        F.close()
    rhs_steps = rng["rhs_steps"] + par["rhs_steps"]
    wall = t3 - t0
    return {"workload": "uneven48: 48 problems, nx in {63,127,255,511} (%s), nu~U[0.5,2], |beta|~U[0,30], "
                        "c~U[0,5], k~U{8..64}, p=k/4, N in {16,32,64}, 32 implicit-Euler steps per slice, T=1; "
                        "FP32 range finder, FP64 Parareal to %g" % (
                            ", ".join("%d x %d^2" % (sum(1 for P in probs if P.nx == g), g) for g in grids), tol),
            "slices": len(slices), "factor_s": t1 - t0, "rsvd_s": t2 - t1, "parareal_s": t3 - t2, "wall_s": wall,
            "rhs_steps_per_s": rhs_steps / wall,
            "range_finder": {"ms": rng["ms"], "launches": rng["launches"], "tflop": rng["flops"] / 1e12,
                             "tflops_per_s": rng["flops"] / rng["ms"] / 1e9},
            "parareal_fine": {"ms": par["ms"], "launches": par["launches"],
                              "algorithmic_GBs": par["bytes"] / max(par["ms"], 1e-9) / 1e6},
            "iters": {"min": int(min(iters)), "max": int(max(iters)), "mean": float(np.mean(iters))},
            "max_err_vs_sequential_fine": float(max(errs)),
            "per_grid": {k: {"problems": v["problems"], "max_err": v["max_err"],
                             "mean_iters": float(np.mean(v["iters"]))} for k, v in per_grid.items()}}


def traffic_from_profile(stem):
    """HBM bytes per range-finder sweep call from the committed rocprofv3
    counter summary of this workload, if it was taken from the current sweep
    sources."""
    from paper_2508_08873_amd import prof_summary
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", stem + ".json")
    if not os.path.exists(path):
        return None, None
    d = json.load(open(path))
    if d.get("source_sha1") != prof_summary.sweep_source_hash() or "traffic_bytes_per_sweep" not in d:
        return None, None
    return d["traffic_bytes_per_sweep"], d


# extra factor store flag of the timed path: the UL set (paired passes)
UL_MASK = [0]


def c1_bench(args, ctx, lrpr, inputs):
    """The 255^2 workload (one shared operator, 64 slices x 32 steps, k = 40,
    p = 10): the whole path per step on --pipelines concurrent pipelines, the
    single-pipeline latency, phase times, the range-finder roofline, the FP64
    side run and the studies.  Returns the result dict."""
    import torch
    UL_MASK[0] = 0 if args.no_ul else lrpr.STORE_UL
    P = inputs.dar255(seed=args.seed)
    prec = args.prec
    # inputs, resident in HBM before the timed region
    # Omega_n: the library's on-device Philox4x32-10 Gaussians, stream n
    Om64 = torch.empty((P.N, P.l, P.n), device="cuda", dtype=torch.float64)
    for s_ in range(P.N):
        ctx.randn(Om64[s_], args.seed, s_)
    u0 = lrpr.colmajor(torch.from_numpy(P.u0().reshape(-1, 1)).to("cuda"))
    f = lrpr.colmajor(torch.from_numpy(P.source().reshape(-1, 1)).to("cuda"))
    fsc = torch.from_numpy(np.concatenate([P.fscale(s) for s in range(1, P.N + 1)])).to("cuda")
    torch.cuda.synchronize()

    def pipeline(prec, steps, warmup):
        """Time `steps` passes of the whole path (after `warmup` untimed ones)
        in one precision of the fine solves and the range finder."""
        fp = 0 if prec == "f64" else 1
        Om = Om64 if prec == "f64" else Om64.to(torch.float32)
        tol = P.tol if prec == "f64" else TOL_F32
        torch.cuda.synchronize()

        def one_step(times, recs, keep):
            ta = time.perf_counter()
            F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt,
                           store_mask=(1 if prec == "f64" else 3) | lrpr.STORE_MIRROR | lrpr.STORE_SPLIT |
                           UL_MASK[0])
            tb = time.perf_counter()
            coarse = ctx.rsvd_build([(F, P.k, P.p, Om[s].t()) for s in range(P.N)], P.m, fp)
            tc = time.perf_counter()
            if recs is not None:
                recs["range"].append(ctx.profile_read())
            out = ctx.parareal_solve(coarse, [F] * P.N, P.m, u0, f, fsc, tol=tol, fine_prec=fp)
            torch.cuda.synchronize()
            td = time.perf_counter()
            if recs is not None:
                recs["parareal"].append(ctx.profile_read())
            times.append((tb - ta, tc - tb, td - tc))
            keep.append((F, coarse))   # released after the timed region
            return out

        def release(keep):
            for F, coarse in keep:
                coarse.close()
                F.close()

        for _ in range(warmup):
            kw = []
            one_step([], None, kw)
            release(kw)
        torch.cuda.synchronize()
        ctx.profile(True)
        times = []
        recs = {"range": [], "parareal": []}
        keep = []
        t0 = time.perf_counter()
        for _ in range(steps):
            out = one_step(times, recs, keep)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.profile(False)
        release(keep)
        return times, recs, t1 - t0, out, tol

    def concurrent(prec, steps, warmup, npipe):
        """`steps` whole-path steps spread round-robin over `npipe` pipelines
        (own context and stream each, one host thread each) after `warmup`
        untimed ones; handles are released after the timed region."""
        fp = 0 if prec == "f64" else 1
        Om = Om64 if prec == "f64" else Om64.to(torch.float32)
        tol = P.tol if prec == "f64" else TOL_F32
        pipes = []
        for _ in range(npipe):
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                pipes.append((st, lrpr.Context(0)))
        torch.cuda.synchronize()

        def run(nsteps):
            counts = [nsteps // npipe + (1 if i < nsteps % npipe else 0) for i in range(npipe)]
            keep = [[] for _ in range(npipe)]
            errs = []

            def worker(i):
                st, c = pipes[i]
                try:
                    with torch.cuda.stream(st):
                        for _ in range(counts[i]):
                            F = c.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt,
                                         store_mask=(1 if prec == "f64" else 3) | lrpr.STORE_MIRROR |
                                         lrpr.STORE_SPLIT | UL_MASK[0])
                            coarse = c.rsvd_build([(F, P.k, P.p, Om[s].t()) for s in range(P.N)], P.m, fp)
                            o = c.parareal_solve(coarse, [F] * P.N, P.m, u0, f, fsc, tol=tol, fine_prec=fp)
                            keep[i].append((F, coarse, o))
                    st.synchronize()
                except Exception as ex:   # reported after the join
                    errs.append(ex)

            th = [threading.Thread(target=worker, args=(i,)) for i in range(npipe)]
            for t in th:
                t.start()
            for t in th:
                t.join()
            if errs:
                raise errs[0]
            return keep

        def release(keep):
            for k in keep:
                for F, coarse, _ in k:
                    coarse.close()
                    F.close()

        release(run(warmup))
        for _, c in pipes:
            c.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        keep = run(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rhs_steps = 0.0
        for _, c in pipes:
            rhs_steps += c.profile_read()["rhs_steps"]
            c.profile(False)
        iters = sorted({o["iters"][0] for k in keep for _, _, o in k})
        release(keep)
        for _, c in pipes:
            c.close()
        return t1 - t0, rhs_steps, iters

    K = args.c1_steps if args.workload == "dar511t" else args.steps
    W = 2 if args.workload == "dar511t" else args.warmup
    times, recs, wall, out, tol = pipeline(prec, K, W)
    t0, t1 = 0.0, wall

    def tot(key, field):
        return sum(r[field] for r in recs[key])

    allp = {k: tot("range", k) + tot("parareal", k) for k in ("ms", "rhs_steps")}
    lat_ms_per_step = (t1 - t0) * 1000.0 / K
    rhs_steps = allp["rhs_steps"] / K
    lat_value = rhs_steps / (lat_ms_per_step / 1000.0)
    if args.pipelines > 1:
        cwall, crhs, citers = concurrent(prec, K, W, args.pipelines)
        ms_per_step = cwall * 1000.0 / K
        value = crhs / cwall
    else:
        ms_per_step, value, citers = lat_ms_per_step, lat_value, [out["iters"][0]]
    # roofline of the dominant kernel: the range-finder sweeps (3200 RHS x 32
    # steps, fine and adjoint; one library call each, timed with the library's
    # events on its stream); the Parareal sweeps (64 RHS) run as partitioned
    # passes, reported by rate below.  The unit of the per-call figures and of
    # `traffic` (HBM bytes, rocprofv3 counters) is one sweep call.
    prof = {k: tot("range", k) for k in ("ms", "launches", "flops", "bytes", "rhs_steps")}
    sweep_s = prof["ms"] / 1000.0
    achieved_tf = prof["flops"] / sweep_s / 1e12 if sweep_s > 0 else 0.0
    achieved_gbs = prof["bytes"] / sweep_s / 1e9 if sweep_s > 0 else 0.0
    peak = PEAK_TFLOPS[prec]
    calls = max(prof["launches"], 1)
    traffic, tsrc = traffic_from_profile("k_sweep_dar255_" + prec)
    roofline = {"bound": "mfma", "achieved": achieved_tf, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved_tf / peak, "traffic": traffic,
                "kernel": ("k_sweep + k_sweep_pair (range-finder band sweeps: 3200 RHS x 32 implicit-Euler steps, "
                           "fine + adjoint; steps alternate L U / U' L', the first and last substitutions run "
                           "alone and the other 62 in 31 pairs)") if UL_MASK[0] else
                          "k_sweep (range-finder band sweeps: 3200 RHS x 32 implicit-Euler steps, fine + adjoint)",
                "sweep_calls": prof["launches"], "avg_sweep_ms": prof["ms"] / calls,
                "algorithmic_flops_per_sweep": prof["flops"] / calls,
                "algorithmic_bytes_per_sweep": prof["bytes"] / calls,
                "traffic_unit": "HBM bytes per sweep call",
                "algorithmic_hbm_GBs": achieved_gbs, "hbm_frac": achieved_gbs / PEAK_HBM_GBS,
                "traffic_source": tsrc["name"] if tsrc else None}
    fac_s = float(np.mean([t[0] for t in times]))
    rsvd_s = float(np.mean([t[1] for t in times]))
    pr_s = float(np.mean([t[2] for t in times]))
    rr = tot("range", "rhs_steps") / max(tot("range", "ms") / 1000.0, 1e-30)
    pr = tot("parareal", "rhs_steps") / max(tot("parareal", "ms") / 1000.0, 1e-30)
    res = {
        "metric": "fine-propagator RHS\u00b7steps/s; rSVD build s; served solve p50/p99 latency",
        "value": value, "unit": "RHS\u00b7steps/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": "dar255: 2D diffusion-advection-reaction, 255x255 interior grid "
                               "(n=65025, b=255), nu=1, beta=(20,10), c=1, T=1, 64 slices x 32 implicit-Euler "
                               "steps, k=40, p=10; step = factor + rSVD build + Parareal to %g" % tol,
                   "rhs_steps_per_step": rhs_steps, "parareal_iters": out["iters"][0],
                   "pipelines": args.pipelines,
                   "range_finder_and_fine_precision": prec,
                   "factorisations": "L U and U' L' (paired passes)" if UL_MASK[0] else "L U",
                   "fp64_steps": "LU, CholeskyQR2 Gram/Cholesky, Jacobi SVD, Parareal correction and residual"},
        "latency": {"pipelines": 1, "ms_per_step": lat_ms_per_step, "value": lat_value,
                    "note": "one pipeline alone, K steps; phase times, rates and the roofline below come from "
                            "this run"},
        "concurrent_parareal_iters": citers,
        "rsvd_build_s": rsvd_s + fac_s, "factor_s": fac_s, "rsvd_only_s": rsvd_s, "parareal_s": pr_s,
        "sweep_kernel_s_per_step": (tot("range", "ms") + tot("parareal", "ms")) / 1000.0 / K,
        "range_finder_sweeps_rhs_steps_per_s": rr, "parareal_sweeps_rhs_steps_per_s": pr,
        "roofline": roofline,
    }
    if prec == "f32" and not args.no_fp64_side:
        # the same pipeline with FP64 fine solves and range finder (to 1e-10)
        t64, r64, w64, o64, tol64 = pipeline("f64", args.fp64_steps, 1)
        rs64 = sum(r["rhs_steps"] for k in r64 for r in r64[k])
        res["fp64_side"] = {"steps": args.fp64_steps, "warmup": 1,
                            "ms_per_step": w64 * 1000.0 / args.fp64_steps, "value": rs64 / w64,
                            "parareal_tol": tol64, "parareal_iters": o64["iters"][0],
                            "factor_s": float(np.mean([t[0] for t in t64])),
                            "rsvd_only_s": float(np.mean([t[1] for t in t64])),
                            "parareal_s": float(np.mean([t[2] for t in t64])),
                            "range_finder_sweeps_rhs_steps_per_s":
                                sum(r["rhs_steps"] for r in r64["range"]) /
                                (sum(r["ms"] for r in r64["range"]) / 1000.0)}
    if not args.no_plain:
        res["range_finder_sweeps_separately"] = fwd_adj_rates(ctx, lrpr, P, prec)
        res["per_step_operators"] = per_step_operators(ctx, lrpr, inputs, prec, args.seed)
        res["neumann_constant_mode"] = neumann_study(ctx, lrpr, args.seed)
        res["fine_steppers"] = stepper_study(ctx, lrpr, P, prec, Om64 if prec == "f64" else Om64.to(torch.float32))
        res["rsvd_variants"] = rsvd_variants(
            ctx, lrpr, P, prec, Om64 if prec == "f64" else Om64.to(torch.float32))
        plain = plain_per_rhs(ctx, lrpr, P)
        res["plain_per_rhs_fp64"] = plain
        if "fp64_side" in res:
            res["batched_vs_plain_per_rhs_fp64_vs_fp64"] = (res["fp64_side"]["range_finder_sweeps_rhs_steps_per_s"] /
                                                            plain["rhs_steps_per_s"])
        res["batched_vs_plain_per_rhs_%s_vs_fp64" % prec] = rr / plain["rhs_steps_per_s"]
    if not args.no_serve:
        res["serve"] = serve_bench(ctx, lrpr, inputs, args.seed, args.serve_rate if args.serve_rate is not None else 4.0,
                                   args.serve_duration if args.serve_duration is not None else 15.0)
    if not args.no_cpu:
        cb, err = cpu_baseline_and_parity(ctx, lrpr, P, prec, args.cpu_cols, args.cpu_steps, args.seed)
        res["cpu_baseline"] = cb
        res["fine_err_vs_oracle"] = err
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the hot path runs on a single MI355X "
              "(multi-GPU sharding is described, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calib:
        copy_calib(args.copy_calib)
        return
    import torch
    from paper_2508_08873_amd import inputs, lrpr

    if args.workload == "dar255":
        res = c1_bench(args, lrpr.Context(0), lrpr, inputs)
        print(json.dumps(res), flush=True)
        return
    if args.workload == "serve3":
        ctx = lrpr.Context(0)
        res = c4_bench(ctx, lrpr, inputs, args)
        sus = res["sustained"]
        print(json.dumps({"metric": "fine-propagator RHS\u00b7steps/s; rSVD build s; served solve p50/p99 latency",
                          "value": res["capacity_solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": 1,
                          "warmup": 0, "ms_per_step": sus["wall_s"] * 1000.0, "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": res["workload"]}, "serve3": res}), flush=True)
        return
    if args.workload == "uneven48":
        ctx = lrpr.Context(0)
        res = c3_bench(ctx, lrpr, inputs, args)
        print(json.dumps({"metric": "fine-propagator RHS\u00b7steps/s; rSVD build s; served solve p50/p99 latency",
                          "value": res["rhs_steps_per_s"], "unit": "RHS\u00b7steps/s", "n_gpus": 1, "steps": 1,
                          "warmup": 0, "ms_per_step": res["wall_s"] * 1000.0, "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
                          "config": {"workload": res["workload"]}, "uneven48": res}), flush=True)
        return
    ctx = lrpr.Context(0)
    P, out, sig, recs, times, wall, tune = c2_bench(ctx, lrpr, args)
    K = args.steps

    def tot(key, field):
        return sum(r[field] for r in recs[key])

    rhs_steps = (tot("range", "rhs_steps") + tot("parareal", "rhs_steps")) / K
    ms_per_step = wall * 1000.0 / K
    value = rhs_steps * K / wall
    # dominant kernel: the range-finder sweeps (one k_sweep launch each way
    # per step: 10240 RHS x 16 steps over 128 factors), FP32 MFMA-bound
    rng = {k: tot("range", k) for k in ("ms", "launches", "flops", "bytes", "rhs_steps")}
    calls = max(rng["launches"], 1)
    sweep_s = rng["ms"] / 1000.0
    achieved = rng["flops"] / sweep_s / 1e12
    traffic, tsrc = traffic_from_profile("k_sweep_dar511t_f32")
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                "frac": achieved / PEAK_TFLOPS["f32"], "traffic": traffic,
                "kernel": "k_sweep (range-finder band sweeps of the 128 slice factors: 10240 RHS x 16 "
                          "implicit-Euler steps in one launch, forward or adjoint)",
                "sweep_calls": rng["launches"], "avg_sweep_ms": rng["ms"] / calls,
                "algorithmic_flops_per_sweep": rng["flops"] / calls,
                "algorithmic_bytes_per_sweep": rng["bytes"] / calls,
                "traffic_unit": "HBM bytes per sweep call",
                "algorithmic_hbm_GBs": rng["bytes"] / sweep_s / 1e9,
                "hbm_frac": rng["bytes"] / sweep_s / 1e9 / PEAK_HBM_GBS,
                "traffic_source": tsrc["name"] if tsrc else None,
                "mfma_busy_frac_counters": tsrc.get("mfma_busy_frac") if tsrc else None}
    # the Parareal sweeps: one RHS per factor, the HBM-bound regime
    par = {k: tot("parareal", k) for k in ("ms", "launches", "flops", "bytes", "rhs_steps")}
    par_s = par["ms"] / 1000.0
    apost = np.array(out["apost"][0])
    res = {
        "metric": "fine-propagator RHS\u00b7steps/s; rSVD build s; served solve p50/p99 latency",
        "value": value, "unit": "RHS\u00b7steps/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "dar511t: 2D diffusion-advection-reaction, 511x511 interior grid (n=261121, b=511), "
                               "nu_n = 1 + 0.5 sin(2 pi t_n) per slice, beta=(20,10), c=1, T=1, 128 slices x 16 "
                               "implicit-Euler steps, k=64, p=16; step = 128 band LUs + rSVD build of all slices + "
                               "Parareal to %g with the per-slice a posteriori bound" % TOL_F32,
                   "rhs_steps_per_step": rhs_steps, "parareal_iters": out["iters"][0],
                   "range_finder_and_fine_precision": "f32",
                   "fp64_steps": "LU, CholeskyQR2 Gram/Cholesky, Jacobi SVD, Parareal correction and residual",
                   "factor_storage": "FP32 tiles, 146 GB for the 128 factors"},
        "rsvd_build_s": float(np.mean([t[0] + t[1] for t in times])),
        "factor_s": float(np.mean([t[0] for t in times])), "rsvd_only_s": float(np.mean([t[1] for t in times])),
        "parareal_s": float(np.mean([t[2] for t in times])),
        "range_finder_sweeps_rhs_steps_per_s": rng["rhs_steps"] / sweep_s,
        "parareal_sweeps": {"rhs_steps_per_s": par["rhs_steps"] / par_s, "calls": par["launches"],
                            "avg_ms": par["ms"] / max(par["launches"], 1),
                            "algorithmic_GBs": par["bytes"] / par_s / 1e9,
                            "hbm_frac": par["bytes"] / par_s / 1e9 / PEAK_HBM_GBS,
                            "note": "one RHS per slice factor (128 factors), FP32; algorithmic bytes = factor "
                                    "read once per step per factor plus the state"},
        "lu_autotune": {"workgroups_per_matrix": tune[0], "chunk_ms": tune[1],
                        "note": "lrpr_autotune_factor before the timed region (one chunk of the 128 factors)"},
        "eps_max_sigma_k1": float(sig[:, P.k].max()), "delta_max_sigma_1": float(sig[:, 0].max()),
        "apost_bound": {"max": float(apost.max()), "slice_1": float(apost[0]), "slice_64": float(apost[63]),
                        "slice_128": float(apost[-1]), "incr": out["incr"][0][:out["iters"][0]]},
        "roofline": roofline,
    }
    if not args.no_cpu:
        res["cpu_baseline"] = c2_cpu_baseline(P, args.c2_cpu_cols, P.m, args.seed)
    if not args.no_side:
        res["dar255"] = c1_bench(args, ctx, lrpr, inputs)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
