"""FP64 CPU oracle for Parareal with low-rank coarse solvers.

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that
the GPU library is checked against.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product code never
does, and it shares no code with the product.

The arithmetic lives in ``lrpr_oracle.c`` (plain loops, FP64, compiled with
``-ffp-contract=off``); this module marshals NumPy arrays into it and adds the
Parareal recursion and the error bounds, written in the paper's notation:

* Parareal iteration and its initialisation: Sec. 2, eq. (def_Parareal).
* Affine fine solver F_n v = F_n' v + b_n with b_n = F_n 0: eq. (F_n_affine).
* Low-rank coarse solver G_n: eq. (spectral_G); its linear part G_n'.
* Randomized SVD: Sec. 2.1 steps 1-6 (in C).
* Neumann boundaries (the variant of the first experiment, Sec. 4; in C), the
  lumped-mass L^2 inner product and the randomized generalized SVD in it
  (eq. svd with the inner product on V; NumPy, Gram-Schmidt in W).
* a priori bound: Thm. 1, eq. (error_bound_eps_delta2);
  a posteriori bound: Thm. 3, eqs. (apost_bound), (apost_bound_sup).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lrpr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblrpr_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle's C code into a shared library (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.ora_assemble_neumann.restype = ctypes.c_int
        lib.ora_assemble_neumann.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        lib.ora_assemble.restype = ctypes.c_int
        lib.ora_assemble.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        lib.ora_band_lu.restype = ctypes.c_int
        lib.ora_band_lu.argtypes = [ctypes.c_int, ctypes.c_int, _dp]
        lib.ora_fine_steps.restype = None
        lib.ora_fine_steps.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_int,
                                       _dp, ctypes.c_long, ctypes.c_int,
                                       _dp, ctypes.c_long, _ip, _dp]
        lib.ora_adjoint_steps.restype = None
        lib.ora_adjoint_steps.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int,
                                          _dp, ctypes.c_long, ctypes.c_int]
        lib.ora_householder_qr.restype = ctypes.c_int
        lib.ora_householder_qr.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_long, _dp, _dp]
        lib.ora_jacobi_svd.restype = ctypes.c_int
        lib.ora_jacobi_svd.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp]
        lib.ora_rsvd.restype = ctypes.c_int
        lib.ora_rsvd.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, _dp, ctypes.c_long, _dp, _dp, _dp]
        lib.ora_rsvd_two_sided.restype = ctypes.c_int
        lib.ora_rsvd_two_sided.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, _dp, _dp, ctypes.c_long, _dp, _dp, _dp]
        lib.ora_rsvd_q.restype = ctypes.c_int
        lib.ora_rsvd_q.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, _dp, ctypes.c_long, _dp, _dp, _dp]
        lib.ora_lowrank_apply.restype = None
        lib.ora_lowrank_apply.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, ctypes.c_int,
                                          _dp, _dp]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _fortran(a):
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def _fortran_copy(a):
    return np.array(a, dtype=np.float64, order="F", copy=True)


# ---------------------------------------------------------------------------
# operator, factor, fine propagator
# ---------------------------------------------------------------------------
class Operator:
    """Implicit-Euler matrix M = I + dt*A of one slice and its band LU.

    A is the finite-difference analogue (first-order upwind advection) of the
    paper's parabolic operator; the fine solver is implicit Euler with m
    steps of size dt per slice (Sec. 4, first paragraph, with finite
    differences in place of finite elements).
    """

    def __init__(self, dim, nx, nu, beta, c, dt, bc="dirichlet"):
        """bc: "dirichlet" (nx interior points per axis, h = 1/(nx+1)) or
        "neumann" (nx points per axis including the boundary, h = 1/(nx-1),
        mirrored ghost points; the variant of the paper's first experiment)."""
        self.dim, self.nx, self.nu, self.c, self.dt = dim, nx, float(nu), float(c), float(dt)
        self.beta = (float(beta[0]), float(beta[1]) if dim == 2 else 0.0)
        self.bc = bc
        self.n = nx if dim == 1 else nx * nx
        self.bw = 1 if dim == 1 else nx
        lib = _load()
        self.band = np.zeros((self.n, 2 * self.bw + 1), dtype=np.float64)
        if bc == "neumann":
            assert nx >= 2
            lib.ora_assemble_neumann(dim, nx, self.nu, self.beta[0], self.beta[1], self.c, self.dt, _p(self.band))
        else:
            assert bc == "dirichlet"
            lib.ora_assemble(dim, nx, self.nu, self.beta[0], self.beta[1], self.c, self.dt, _p(self.band))
        self.lu = self.band.copy()
        info = lib.ora_band_lu(self.n, self.bw, _p(self.lu))
        if info != 0:
            raise ArithmeticError("zero pivot at row %d" % (info - 1))

    def dense(self):
        """Dense M (for tiny test grids only)."""
        n, b = self.n, self.bw
        M = np.zeros((n, n))
        for i in range(n):
            for j in range(max(0, i - b), min(n, i + b + 1)):
                M[i, j] = self.band[i, j - i + b]
        return M

    def dense_lu(self):
        """Dense (L, U) of the band LU (tiny grids only)."""
        n, b = self.n, self.bw
        L, U = np.eye(n), np.zeros((n, n))
        for i in range(n):
            for j in range(max(0, i - b), min(n, i + b + 1)):
                if j < i:
                    L[i, j] = self.lu[i, j - i + b]
                else:
                    U[i, j] = self.lu[i, j - i + b]
        return L, U

    def fine(self, X, m, f=None, fcol=None, fscale=None):
        """m implicit-Euler steps for every column of X (n x w), returns a new array.

        Column c gets the source fscale[c, j] * f[:, fcol[c]] at step j (evaluated
        at the step's end time); without f the map is T = M^{-m}.
        """
        X = _fortran_copy(X)
        if X.ndim == 1:
            X = X.reshape(-1, 1, order="F")
        n, w = X.shape
        assert n == self.n
        fp = fc = fs = None
        ldf = 0
        if f is not None:
            f = _fortran(f)
            if f.ndim == 1:
                f = f.reshape(-1, 1, order="F")
            ldf = f.shape[0]
            fcol = np.ascontiguousarray(np.zeros(w, np.int32) if fcol is None else fcol, dtype=np.int32)
            fc = fcol.ctypes.data_as(_ip)
            fp = _p(f)
            if fscale is not None:
                fscale = np.ascontiguousarray(np.broadcast_to(np.asarray(fscale, np.float64), (w, m)))
                fs = _p(fscale)
        _load().ora_fine_steps(self.n, self.bw, _p(self.lu), self.dt, m, _p(X), n, w, fp, ldf, fc, fs)
        return X

    def adjoint(self, X, m):
        """X <- (M^T)^{-m} X, the adjoint of the source-free fine propagator."""
        X = _fortran_copy(X)
        if X.ndim == 1:
            X = X.reshape(-1, 1, order="F")
        n, w = X.shape
        _load().ora_adjoint_steps(self.n, self.bw, _p(self.lu), m, _p(X), n, w)
        return X


# ---------------------------------------------------------------------------
# SDIRK fine steppers (the Butcher tableaus of the paper's study of the time
# discretisation, Sec. 4 "Effect of time discretization")
# ---------------------------------------------------------------------------
GAMMA_L = (2.0 - 2.0 ** 0.5) / 2.0
TABLEAUS = {
    # c, a (lower triangular), b
    "sdirk2": ((1.0, 0.0), ((1.0, 0.0), (-1.0, 1.0)), (0.5, 0.5)),
    "sdirk2l": ((GAMMA_L, 1.0), ((GAMMA_L, 0.0), (1.0 - GAMMA_L, GAMMA_L)), (1.0 - GAMMA_L, GAMMA_L)),
}


class Stepper:
    """m steps of a two-stage SDIRK method for u' = -A u + f(t), stage by
    stage from the tableau: with t the step's start,
        (I + dt a_ii A) k_i = -A (u + dt sum_{l<i} a_il k_l) + f(t + c_i dt),
        u_new = u + dt sum_i b_i k_i.
    The diagonal entries are equal, so every stage solves with the one band
    LU of I + a_11 dt A; A v comes from that matrix, A v = (M v - v) / (a_11 dt).
    The source of column c at stage i of step j is fscale[c, 2j + i] f[:, fcol[c]].
    The linear map of a step is a rational function of A, so its adjoint is
    the same recurrence with A^T and M^T (adjoint)."""

    def __init__(self, method, dim, nx, nu, beta, c, dt):
        self.method = method
        self.cs, self.a, self.b = TABLEAUS[method]
        self.dt = float(dt)
        self.g = self.a[0][0]
        self.stage = Operator(dim, nx, nu, beta, c, self.g * self.dt)
        self.n = self.stage.n

    def _A(self, V, transpose=False):
        st, b, n = self.stage, self.stage.bw, self.stage.n
        out = np.zeros_like(V)
        for d in range(-b, b + 1):
            if transpose:   # (M^T v)_i = sum_d M[i - d, i] v[i - d]
                lo, hi = max(0, d), min(n, n + d)
                out[lo:hi] += st.band[lo - d:hi - d, d + b][:, None] * V[lo - d:hi - d]
            else:           # (M v)_i = sum_d M[i, i + d] v[i + d]
                lo, hi = max(0, -d), min(n, n - d)
                out[lo:hi] += st.band[lo:hi, d + b][:, None] * V[lo + d:hi + d]
        return (out - V) / (self.g * self.dt)

    def _solve(self, V, transpose=False):
        return self.stage.adjoint(V, 1) if transpose else self.stage.fine(V, 1)

    def _run(self, X, m, transpose, f=None, fcol=None, fscale=None):
        X = np.array(X, dtype=np.float64, copy=True)
        if X.ndim == 1:
            X = X.reshape(-1, 1)
        w = X.shape[1]
        if f is not None:
            f = np.asarray(f, dtype=np.float64)
            if f.ndim == 1:
                f = f.reshape(-1, 1)
            fcol = np.zeros(w, dtype=np.int64) if fcol is None else np.asarray(fcol)
            F = f[:, fcol]
            fscale = np.ones((w, 2 * m)) if fscale is None else np.broadcast_to(np.asarray(fscale, np.float64), (w, 2 * m))
        for j in range(m):
            K = []
            for i in range(2):
                Ui = X.copy()
                for l in range(i):
                    Ui += self.dt * self.a[i][l] * K[l]
                rhs = -self._A(Ui, transpose)
                if f is not None:
                    rhs += F * fscale[:, 2 * j + i][None, :]
                K.append(self._solve(rhs, transpose))
            for i in range(2):
                X += self.dt * self.b[i] * K[i]
        return X

    def fine(self, X, m, f=None, fcol=None, fscale=None):
        return self._run(X, m, False, f, fcol, fscale)

    def adjoint(self, X, m):
        return self._run(X, m, True)


class StepSequence:
    """m implicit-Euler steps with per-step operators, step j solving with
    M_j = I + dt_j A_j (time-dependent coefficients inside a slice):
    T = M_m^{-1} ... M_1^{-1}; the adjoint is T^T = M_1^{-T} ... M_m^{-T}.
    The source of column c at step j is fscale[c, j] f[:, fcol[c]]."""

    def __init__(self, ops):
        self.ops = [Operator(**o) for o in ops]
        self.n = self.ops[0].n

    def fine(self, X, m, f=None, fcol=None, fscale=None):
        X = np.array(X, dtype=np.float64, copy=True)
        if X.ndim == 1:
            X = X.reshape(-1, 1)
        w = X.shape[1]
        if fscale is not None:
            fscale = np.broadcast_to(np.asarray(fscale, np.float64), (w, m))
        for j in range(m):
            X = self.ops[j].fine(X, 1, f, fcol, None if fscale is None else fscale[:, j:j + 1])
        return X

    def adjoint(self, X, m):
        X = np.array(X, dtype=np.float64, copy=True)
        for j in reversed(range(m)):
            X = self.ops[j].adjoint(X, 1)
        return X


def householder_qr(Y):
    Y = _fortran(Y)
    n, l = Y.shape
    Q = np.zeros((n, l), order="F")
    R = np.zeros((l, l), order="F")
    _load().ora_householder_qr(n, l, _p(Y), n, _p(Q), _p(R))
    return Q, R


def jacobi_svd(M):
    M = _fortran(M)
    l = M.shape[0]
    U = np.zeros((l, l), order="F")
    V = np.zeros((l, l), order="F")
    S = np.zeros(l)
    sweeps = _load().ora_jacobi_svd(l, _p(M), _p(U), _p(S), _p(V))
    if sweeps < 0:
        raise ArithmeticError("Jacobi SVD did not converge")
    return U, S, V


def rsvd(op: Operator, m: int, k: int, p: int, Omega, q: int = 0):
    """Randomized SVD of T = M^{-m} (Sec. 2.1), with q power iterations
    (range space span (T T^T)^q T Omega).  Returns (Uk, S_all, Vk)."""
    Omega = _fortran(Omega)
    n, l = Omega.shape
    assert l == k + p and n == op.n and q >= 0
    Uk = np.zeros((n, k), order="F")
    Vk = np.zeros((n, k), order="F")
    S = np.zeros(l)
    sw = _load().ora_rsvd_q(n, op.bw, _p(op.lu), m, k, p, q, _p(Omega), n, _p(Uk), _p(S), _p(Vk))
    if sw < 0:
        raise ArithmeticError("Jacobi SVD did not converge")
    return Uk, S, Vk


def rsvd_general(op, m: int, k: int, p: int, Omega):
    """Randomized SVD (Sec. 2.1, steps 1-6) through the operator's own fine
    and adjoint maps (for the SDIRK steppers): Y = T Omega, Y = Q R, Z = T^T Q,
    Z = Qz Rz, Rz^T = Uh diag(S) Vh^T, Uk = Q Uh[:, :k], Vk = Qz Vh[:, :k], the
    pairs signed as in rsvd.  Returns (Uk, S_all, Vk)."""
    Y = op.fine(np.asarray(Omega, np.float64), m)
    Q, _ = householder_qr(Y)
    Z = op.adjoint(Q, m)
    Qz, Rz = householder_qr(Z)
    Uh, S, Vh = jacobi_svd(np.asfortranarray(Rz.T))
    Uk = Q @ Uh[:, :k]
    Vk = Qz @ Vh[:, :k]
    for r in range(k):
        im = int(np.argmax(np.abs(Uk[:, r])))
        if Uk[im, r] < 0:
            Uk[:, r] *= -1.0
            Vk[:, r] *= -1.0
    return Uk, S, Vk


def rsvd_two_sided(op: Operator, m: int, k: int, p: int, Omega, Psi):
    """Randomized SVD with the adjoint on independent test vectors Psi
    (Sec. 2.2): T ~ Q (Psi^T Q)^{-1} (T^T Psi)^T with Q = orth(T Omega),
    truncated to rank k.  Returns (Uk, S_all, Vk)."""
    Omega, Psi = _fortran(Omega), _fortran(Psi)
    n, l = Omega.shape
    assert l == k + p and n == op.n and Psi.shape == (n, l)
    Uk = np.zeros((n, k), order="F")
    Vk = np.zeros((n, k), order="F")
    S = np.zeros(l)
    sw = _load().ora_rsvd_two_sided(n, op.bw, _p(op.lu), m, k, p, _p(Omega), _p(Psi), n, _p(Uk), _p(S), _p(Vk))
    if sw == -2:
        raise ArithmeticError("Psi^T Q is singular")
    if sw < 0:
        raise ArithmeticError("Jacobi SVD did not converge")
    return Uk, S, Vk


def mass_weights(dim, nx, bc="dirichlet"):
    """Lumped (trapezoidal) mass matrix of the grid, the diagonal weights of
    the discrete L^2 inner product (u, v)_W = sum_i w_i u_i v_i.  Dirichlet:
    every unknown is interior, w = h^dim.  Neumann: the boundary points carry
    half the weight per axis (w_i = h/2 at both ends), so sum(w) = 1."""
    if bc == "neumann":
        h = 1.0 / (nx - 1)
        w1 = np.full(nx, h)
        w1[0] = w1[-1] = 0.5 * h
    else:
        h = 1.0 / (nx + 1)
        w1 = np.full(nx, h)
    if dim == 1:
        return w1
    return np.kron(w1, w1)   # index i + nx*j: w_i * w_j


def orth_weighted(Y, w):
    """Orthonormal basis of range(Y) in (u, v)_W (modified Gram-Schmidt, two
    passes): Y = Q R with Q^T W Q = I, R upper triangular."""
    Y = np.array(Y, dtype=np.float64)
    n, l = Y.shape
    Q = np.zeros((n, l))
    R = np.zeros((l, l))
    for j in range(l):
        v = Y[:, j].copy()
        for _ in range(2):
            for i in range(j):
                c = np.dot(Q[:, i] * w, v)
                R[i, j] += c
                v -= c * Q[:, i]
        R[j, j] = math.sqrt(np.dot(v * w, v))
        Q[:, j] = v / R[j, j]
    return Q, R


def rsvd_weighted(op, m, k, p, Omega, w):
    """Randomized generalized SVD of T = F_n' in the inner product (u, v)_W
    (eq. svd with the inner product on V; Sec. 2.1 steps 1-6 with every inner
    product and the adjoint taken in W):
      Y = T Omega;  Y = Q R  (Q^T W Q = I);
      Z = T^* Q with the W-adjoint T^* = W^{-1} T^T W;  Z = Qz Rz;
      Rz^T = Uh diag(S) Vh^T;  psi = Q Uh[:, :k],  phi = Qz Vh[:, :k],
    so that T v ~ sum_r psi_r S_r (phi_r, v)_W.  Returns (Uk, S_all, Vk) with
    Uk = psi and Vk = W phi (then G_n' v = Uk (S .* (Vk^T v)) as for the
    Euclidean build); pairs signed as in rsvd."""
    w = np.asarray(w, np.float64)
    Y = op.fine(np.asarray(Omega, np.float64), m)
    Q, _ = orth_weighted(Y, w)
    Z = op.adjoint(Q * w[:, None], m) / w[:, None]
    Qz, Rz = orth_weighted(Z, w)
    Uh, S, Vht = np.linalg.svd(Rz.T)
    Uk = Q @ Uh[:, :k]
    Phi = Qz @ Vht.T[:, :k]
    for r in range(k):
        im = int(np.argmax(np.abs(Uk[:, r])))
        if Uk[im, r] < 0:
            Uk[:, r] *= -1.0
            Phi[:, r] *= -1.0
    return Uk, S, Phi * w[:, None]


def neumann_eigenvalues(dim, nx, nu, c):
    """Eigenvalues of A for the Neumann operator without advection: the
    mirrored-ghost Laplacian has eigenvectors cos(j pi x_i) with eigenvalues
    (4/h^2) sin^2(j pi h / 2), j = 0..nx-1, h = 1/(nx-1); in 2D the sums
    over both axes."""
    h = 1.0 / (nx - 1)
    lam = 4.0 / (h * h) * np.sin(np.arange(nx) * math.pi * h / 2.0) ** 2
    if dim == 2:
        lam = (lam[:, None] + lam[None, :]).ravel()
    return nu * lam + c


def lowrank_apply(Uk, S, Vk, V):
    """G_n' V = Uk (S .* (Vk^T V)) column by column."""
    Uk, Vk, V = _fortran(Uk), _fortran(Vk), _fortran(V)
    if V.ndim == 1:
        V = V.reshape(-1, 1, order="F")
    n, k = Uk.shape
    w = V.shape[1]
    S = np.ascontiguousarray(S[:k], dtype=np.float64)
    out = np.zeros((n, w), order="F")
    _load().ora_lowrank_apply(n, k, _p(Uk), _p(S), _p(Vk), w, _p(V), _p(out))
    return out


# ---------------------------------------------------------------------------
# Parareal (Sec. 2) and bounds (Sec. 3)
# ---------------------------------------------------------------------------
class Slice:
    """One Parareal interval [t_{n-1}, t_n]: its fine solver F_n (operator, m
    steps, source f with per-step time factors) and, once built, the coarse
    factors (Uk, S, Vk) and b_n = F_n 0."""

    def __init__(self, op: Operator, m: int, f=None, fscale=None):
        self.op, self.m, self.f, self.fscale = op, m, f, fscale
        self.Uk = self.S = self.Vk = None
        self.b = None

    def F(self, v):
        """Affine fine solver F_n v (eq. F_n_affine)."""
        if self.f is None:
            return self.op.fine(v, self.m)[:, 0]
        return self.op.fine(v, self.m, self.f, None, self.fscale)[:, 0]

    def Fp(self, v):
        """Linear part F_n' = T_n."""
        return self.op.fine(v, self.m)[:, 0]

    def Gp(self, v):
        """Linear part G_n' of the coarse solver."""
        if self.Uk is None or self.Uk.shape[1] == 0:
            return np.zeros(self.op.n)
        return lowrank_apply(self.Uk, self.S, self.Vk, v)[:, 0]


def fine_all(slices, vs):
    """[F_n v_n for every slice n]: the fine solves of one Parareal
    iteration, which are independent across slices (Sec. 2.2).  Consecutive
    slices with the same operator, step count and source run as the columns
    of one call (each column's arithmetic is that of a call of its own)."""
    out = [None] * len(slices)
    i = 0
    while i < len(slices):
        s = slices[i]
        j = i + 1
        if isinstance(getattr(s, "op", None), Operator):
            while (j < len(slices) and getattr(slices[j], "op", None) is s.op and slices[j].m == s.m
                   and slices[j].f is s.f):
                j += 1
        if j == i + 1:
            out[i] = s.F(vs[i])
        else:
            X = np.stack([np.asarray(vs[q], np.float64) for q in range(i, j)], axis=1)
            if s.f is None:
                Y = s.op.fine(X, s.m)
            else:
                fsc = None
                if s.fscale is not None:
                    fsc = np.stack([np.broadcast_to(np.asarray(slices[q].fscale, np.float64), (s.m,))
                                    for q in range(i, j)])
                else:
                    fsc = np.ones((j - i, s.m))
                Y = s.op.fine(X, s.m, s.f, None, fsc)
            for q in range(i, j):
                out[q] = Y[:, q - i].copy()
        i = j
    return out


def build_coarse(slices, k, p, omegas):
    """Set up all coarse solvers: rSVD of every F_n' and b_n = F_n 0."""
    for s, om in zip(slices, omegas):
        if k + p > 0:
            build = rsvd if isinstance(s.op, Operator) else rsvd_general
            s.Uk, s.S, s.Vk = build(s.op, s.m, k, p, om)
        else:
            s.Uk = np.zeros((s.op.n, 0))
            s.Vk = np.zeros((s.op.n, 0))
            s.S = np.zeros(0)
    for s, b in zip(slices, fine_all(slices, [np.zeros(s.op.n) for s in slices])):
        s.b = b


def sequential(slices, u0):
    """Reference trajectory u_n = F_n u_{n-1} (Sec. 2, first display)."""
    u = [np.asarray(u0, np.float64).copy()]
    for s in slices:
        u.append(s.F(u[-1]))
    return np.array(u)


def parareal(slices, u0, tol, max_iter=None):
    """Parareal with low-rank coarse solvers, eq. (def_Parareal).

    u^k_0 = u0;  u^0_n = G_n u^0_{n-1} = G_n' u^0_{n-1} + b_n;
    u^{k+1}_n = F_n u^k_{n-1} + G_n' u^{k+1}_{n-1} - G_n' u^k_{n-1}.
    The b_n cancel in the correction (Remark on the affine part), so the
    linear part G_n' is used there and G_n' u^k_{n-1} is kept from the
    previous sweep.  Stops when max_n ||u^{k+1}_n - u^k_n||_2 < tol or after
    N iterations (where the iteration is exact).

    Returns dict: iterates (list of (N+1) x n arrays, u^0..u^K), incr (list),
    iters (K).
    """
    N = len(slices)
    if max_iter is None:
        max_iter = N
    u0 = np.asarray(u0, np.float64)
    cur = [u0.copy()]
    gold = [None]
    for n in range(1, N + 1):
        gp = slices[n - 1].Gp(cur[n - 1])
        gold.append(gp)
        cur.append(gp + slices[n - 1].b)
    iterates = [np.array(cur)]
    incrs = []
    k = 0
    while k < max_iter:
        Fu = [None] + fine_all(slices, cur[:N])
        new = [u0.copy()]
        gnew = [None]
        for n in range(1, N + 1):
            gp = slices[n - 1].Gp(new[n - 1])
            gnew.append(gp)
            new.append(Fu[n] + gp - gold[n])
        incr = max(float(np.linalg.norm(new[n] - cur[n])) for n in range(1, N + 1))
        incrs.append(incr)
        cur, gold = new, gnew
        iterates.append(np.array(cur))
        k += 1
        if incr < tol or k >= N:
            break
    return {"iterates": iterates, "incr": incrs, "iters": k}


def bound_constants(slices, k):
    """delta = max_n sigma_{n,1}, eps = max_n sigma_{n,k+1} (Thm. 1, eq.
    bounds_delta_eps); sigma_{n,k+1} is taken from the oversampled values."""
    delta = max(float(s.S[0]) for s in slices)
    eps = max(float(s.S[k]) if len(s.S) > k else 0.0 for s in slices)
    return delta, eps


def apriori_bound(delta, eps, bnorms, k, n):
    """Thm. 1, eq. (error_bound_eps_delta2):
    ||e^k_n|| <= 2 eps^k sum_{m=0}^{n-k-1} C(n-m, k) delta^{n-m-k} ||b_m||,
    with b_0 = u_0."""
    s = 0.0
    for m in range(0, n - k):
        s += math.comb(n - m, k) * delta ** (n - m - k) * bnorms[m]
    return 2.0 * eps ** k * s


def apost_bound(delta, eps, incr_norms):
    """Thm. 3, eq. (apost_bound): for n = 1..N,
    ||e^k_n|| <= eps sum_{m=1}^{n-1} delta^{n-m-1} ||u^k_m - u^{k-1}_m||.
    incr_norms[m-1] = ||u^k_m - u^{k-1}_m|| for m = 1..N.  Returns N values."""
    N = len(incr_norms)
    out = []
    for n in range(1, N + 1):
        s = 0.0
        for m in range(1, n):
            s += delta ** (n - m - 1) * incr_norms[m - 1]
        out.append(eps * s)
    return np.array(out)
