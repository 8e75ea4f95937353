"""Seeded synthetic inputs for the low-rank Parareal workloads.

This module holds problem definitions and random draws only: grid
coordinates, initial values, source terms and their time factors, Gaussian
test matrices.  It contains none of the method's arithmetic (no operator
assembly, no solves, no SVD), so both the GPU library's tests and the CPU
oracle can take their inputs from it.

Workloads (finite-difference, implicit-Euler analogues of the paper's
parabolic test problems, Sec. 4):

* ``heat1d``   1D heat equation, n=255 interior points, 16 slices x 64 steps,
               k=10, p=5, u0 = sin(pi x) + 0.1*noise, f = sin(2 pi x) cos(2 pi t).
* ``dar255``   2D diffusion-advection-reaction on a 255^2 interior grid,
               nu=1, beta=(20,10), c=1, 64 slices x 32 steps, k=40, p=10,
               f = 4 Gaussian bumps, u0 = 8x8-mode sine field.
* ``dar511t``  511^2 grid, nu_n = 1 + 0.5 sin(2 pi t_n) per slice, 128 slices
               x 16 steps, k=64, p=16.
* ``uneven48`` 48 independent problems of uneven grid and rank.
* ``serve3``   3 operators (127^2, 255^2, 511^2) with per-request u0 and f.

Random streams are derived from ``numpy.random.SeedSequence([seed, stream,
*idx])`` so that every array can be regenerated independently.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

STREAMS = {"omega": 1, "u0": 2, "f": 3, "problem": 4, "arrivals": 5, "request": 6, "psi": 7}


def rng(seed: int, stream: str, *idx: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), STREAMS[stream], *[int(i) for i in idx]]))


@dataclass
class Problem:
    """One parabolic problem on [0, T] cut into N slices of m steps each."""
    name: str
    dim: int
    nx: int
    nu: float
    beta: tuple
    c: float
    T: float
    N: int
    m: int
    k: int
    p: int
    tol: float = 1e-10
    src_kind: str = "bumps"        # "sin2pi" (1D heat) or "bumps"
    nbumps: int = 4
    u0_kind: str = "fourier"       # "sin_noise" (1D) or "fourier"
    nu_of_t: bool = False          # nu_n = 1 + 0.5 sin(2 pi t_n) per slice
    seed: int = 0
    pid: int = 0                   # problem index inside a batch (random streams)
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nx if self.dim == 1 else self.nx * self.nx

    @property
    def bw(self) -> int:
        return 1 if self.dim == 1 else self.nx

    @property
    def dt(self) -> float:
        return self.T / (self.N * self.m)

    @property
    def l(self) -> int:
        return self.k + self.p

    def t(self, n: int) -> float:
        """t_n = n T / N (uniform partition)."""
        return n * self.T / self.N

    def nu_slice(self, n: int) -> float:
        """Diffusion coefficient of slice n (1-based); time-dependent problems
        freeze nu at the slice's right end point t_n."""
        if self.nu_of_t:
            return 1.0 + 0.5 * math.sin(2.0 * math.pi * self.t(n))
        return self.nu

    def op_params(self, n: int = 1) -> dict:
        return dict(dim=self.dim, nx=self.nx, nu=self.nu_slice(n), beta=self.beta, c=self.c, dt=self.dt)

    # -- grid ---------------------------------------------------------------
    def grid(self):
        h = 1.0 / (self.nx + 1)
        x = h * np.arange(1, self.nx + 1)
        if self.dim == 1:
            return (x,)
        X, Y = np.meshgrid(x, x, indexing="xy")          # index r = i + nx*j
        return X.reshape(-1), Y.reshape(-1)

    # -- data ---------------------------------------------------------------
    def u0(self, req: int = 0) -> np.ndarray:
        g = self.grid()
        if self.u0_kind == "sin_noise":
            r = rng(self.seed, "u0", self.pid, req)
            return np.sin(math.pi * g[0]) + 0.1 * r.standard_normal(self.n)
        r = rng(self.seed, "u0", self.pid, req)
        a = r.standard_normal((8, 8))
        x, y = g
        u = np.zeros(self.n)
        for j in range(1, 9):
            sx = np.sin(j * math.pi * x)
            for l in range(1, 9):
                u += a[j - 1, l - 1] / (j * l) * sx * np.sin(l * math.pi * y)
        return u

    def source(self, req: int = 0) -> np.ndarray:
        """Spatial part f(x) of the separable source f(x) phi(t)."""
        g = self.grid()
        if self.src_kind == "sin2pi":
            return np.sin(2.0 * math.pi * g[0])
        r = rng(self.seed, "f", self.pid, req)
        nb = self.nbumps if req == 0 or "bumps_per_req" not in self.extra else int(r.integers(1, 7))
        cen = r.uniform(0.2, 0.8, size=(nb, 2))
        amp = r.standard_normal(nb)
        x, y = g
        f = np.zeros(self.n)
        for q in range(nb):
            f += amp[q] * np.exp(-((x - cen[q, 0]) ** 2 + (y - cen[q, 1]) ** 2) / (2.0 * 0.05 ** 2))
        return f

    def phi(self, t):
        """Time factor phi(t) of the source."""
        if self.src_kind == "sin2pi":
            return np.cos(2.0 * math.pi * np.asarray(t))
        return np.ones_like(np.asarray(t, dtype=np.float64))

    def fscale(self, n: int) -> np.ndarray:
        """phi at the end time of each implicit-Euler step of slice n (1-based):
        phi(t_{n-1} + (j+1) dt), j = 0..m-1."""
        t = self.t(n - 1) + (np.arange(self.m) + 1) * self.dt
        return self.phi(t)

    def step_ops(self, n: int) -> list:
        """Operator parameters of every implicit-Euler step of slice n
        (1-based) for per-step operators: nu at the step's end time
        t_{n-1} + (j+1) dt when nu depends on t, else the slice's."""
        out = []
        for j in range(self.m):
            d = self.op_params(n)
            if self.nu_of_t:
                t = self.t(n - 1) + (j + 1) * self.dt
                d["nu"] = 1.0 + 0.5 * math.sin(2.0 * math.pi * t)
            out.append(d)
        return out

    def fscale_stages(self, n: int, cs) -> np.ndarray:
        """phi at the stage times of a two-stage stepper with abscissae cs in
        slice n: phi(t_{n-1} + (j + c_i) dt), j = 0..m-1, i = 0, 1 (step order)."""
        j = np.repeat(np.arange(self.m), len(cs))
        c = np.tile(np.asarray(cs, np.float64), self.m)
        return self.phi(self.t(n - 1) + (j + c) * self.dt)

    def omega(self, n: int, dtype=np.float64) -> np.ndarray:
        """Gaussian test matrix Omega_n (n x l, column-major) of slice n."""
        r = rng(self.seed, "omega", self.pid, n)
        return np.asfortranarray(r.standard_normal((self.l, self.n)).T).astype(dtype)

    def psi(self, n: int, dtype=np.float64) -> np.ndarray:
        """Second Gaussian test matrix Psi_n (n x l), independent of Omega_n,
        for the adjoint evaluations of the two-sided build."""
        r = rng(self.seed, "psi", self.pid, n)
        return np.asfortranarray(r.standard_normal((self.l, self.n)).T).astype(dtype)


def heat1d(seed: int = 0, **kw) -> Problem:
    return Problem(name="heat1d", dim=1, nx=255, nu=1.0, beta=(0.0, 0.0), c=0.0, T=1.0, N=16, m=64,
                   k=10, p=5, tol=1e-10, src_kind="sin2pi", u0_kind="sin_noise", seed=seed, **kw)


def dar255(seed: int = 0, **kw) -> Problem:
    d = dict(name="dar255", dim=2, nx=255, nu=1.0, beta=(20.0, 10.0), c=1.0, T=1.0, N=64, m=32,
             k=40, p=10, tol=1e-10, seed=seed)
    d.update(kw)
    return Problem(**d)


def dar511t(seed: int = 0, **kw) -> Problem:
    d = dict(name="dar511t", dim=2, nx=511, nu=1.0, beta=(20.0, 10.0), c=1.0, T=1.0, N=128, m=16,
             k=64, p=16, tol=1e-10, nu_of_t=True, seed=seed)
    d.update(kw)
    return Problem(**d)


def dar127s(seed: int = 0, **kw) -> Problem:
    """Per-step operators: 127^2 grid, nu(t) = 1 + 0.5 sin(2 pi t) changing every
    implicit-Euler step (one factor per step), 16 slices x 8 steps, k = 20, p = 5."""
    d = dict(name="dar127s", dim=2, nx=127, nu=1.0, beta=(20.0, 10.0), c=1.0, T=1.0, N=16, m=8,
             k=20, p=5, tol=1e-10, nu_of_t=True, seed=seed)
    d.update(kw)
    return Problem(**d)


def uneven48(seed: int = 0, count: int = 48) -> list:
    """48 problems drawn in order: nx in {63,127,255,511}, nu ~ U[0.5,2],
    |beta| ~ U[0,30], theta ~ U[0,2pi), c ~ U[0,5], k ~ U{8..64}, p = floor(k/4),
    N in {16,32,64}; m = 32 steps per slice, T = 1."""
    r = rng(seed, "problem", 0)
    out = []
    for i in range(count):
        nx = int(r.choice([63, 127, 255, 511]))
        nu = float(r.uniform(0.5, 2.0))
        bmag = float(r.uniform(0.0, 30.0))
        th = float(r.uniform(0.0, 2.0 * math.pi))
        c = float(r.uniform(0.0, 5.0))
        k = int(r.integers(8, 65))
        N = int(r.choice([16, 32, 64]))
        out.append(Problem(name="uneven48_%02d" % i, dim=2, nx=nx, nu=nu,
                           beta=(bmag * math.cos(th), bmag * math.sin(th)), c=c, T=1.0, N=N, m=32,
                           k=k, p=k // 4, seed=seed, pid=i + 1))
    return out


def serve3(seed: int = 0) -> list:
    """Three serving operators: 127^2, 255^2, 511^2; nu=1, beta=(10,5), c=1,
    N=64 slices x 32 steps, k=48, p=12, tolerance 1e-8."""
    return [Problem(name="serve%d" % nx, dim=2, nx=nx, nu=1.0, beta=(10.0, 5.0), c=1.0, T=1.0, N=64,
                    m=32, k=48, p=12, tol=1e-8, seed=seed, pid=100 + i, extra={"bumps_per_req": True})
            for i, nx in enumerate((127, 255, 511))]


def tiny2d(nx: int = 15, N: int = 6, m: int = 4, k: int = 6, p: int = 3, seed: int = 0, **kw) -> Problem:
    """Small 2D problem for CPU tests and GPU parity at oracle-friendly sizes."""
    d = dict(name="tiny2d_%d" % nx, dim=2, nx=nx, nu=1.0, beta=(20.0, 10.0), c=1.0, T=1.0 / 16.0, N=N,
             m=m, k=k, p=p, tol=1e-12, seed=seed)
    d.update(kw)
    return Problem(**d)


def arrivals(seed: int = 0, rate: float = 200.0, duration: float = 60.0) -> np.ndarray:
    """Poisson arrival times (exponential gaps) for the serving workload."""
    r = rng(seed, "arrivals", 0)
    gaps = r.exponential(1.0 / rate, size=int(rate * duration * 1.5) + 16)
    t = np.cumsum(gaps)
    return t[t < duration]
