"""Thin ctypes binding of the lrpr C ABI (include/lrpr.h).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the computation runs in the library's HIP
kernels.  Loading fails loudly if ``liblrpr.so`` has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblrpr.so")

LRPR_F64, LRPR_F32 = 0, 1
STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_NOMEM", 3: "ERR_ZERO_PIVOT", 4: "ERR_QR_BREAKDOWN",
          5: "ERR_NOCONV", 6: "ERR_NONFINITE", 7: "ERR_HIP"}
EXPORTS = ["lrpr_ctx_create", "lrpr_ctx_destroy", "lrpr_ctx_set_stream", "lrpr_last_error",
           "lrpr_ctx_release_workspaces", "lrpr_tune_set", "lrpr_tune_get", "lrpr_autotune_factor",
           "lrpr_device_trim",
           "lrpr_factor", "lrpr_factor_stepper", "lrpr_factor_sequence", "lrpr_factor_many", "lrpr_factor_destroy",
           "lrpr_factor_info", "lrpr_factor_copy_lu", "lrpr_factor_copy_tiles",
           "lrpr_fine_step_batched", "lrpr_adjoint_step_batched", "lrpr_rsvd_build", "lrpr_rsvd_build_q",
           "lrpr_rsvd_build_two_sided", "lrpr_rsvd_build_w", "lrpr_coarse_from_factors", "lrpr_mass_weights",
           "lrpr_coarse_destroy", "lrpr_coarse_view", "lrpr_coarse_get", "lrpr_coarse_apply",
           "lrpr_coarse_apply_noalloc",
           "lrpr_parareal_solve", "lrpr_parareal_solve_many",
           "lrpr_profile_enable", "lrpr_profile_read", "lrpr_randn",
           "lrpr_server_create", "lrpr_server_destroy", "lrpr_server_submit", "lrpr_server_progress",
           "lrpr_server_stats", "lrpr_server_last_error"]


# lrpr_tune_set parameters
TUNE_LU_WGS, TUNE_LU_BUDGET, TUNE_PARAREAL_GRAPH, TUNE_SWEEP_GROUPS, TUNE_RSVD_BUDGET = 1, 2, 3, 4, 5
# lrpr_factor store_mask bits (include/lrpr.h)
STORE_F64, STORE_F32, STORE_MIRROR, STORE_SPLIT, STORE_UL = 1, 2, 4, 8, 16
# lrpr_factor_stepper steppers
STEP_EULER, STEP_SDIRK2, STEP_SDIRK2L, STEP_SEQUENCE = 0, 1, 2, 3
# lrpr_op_desc boundary conditions
BC_DIRICHLET, BC_NEUMANN = 0, 1


class LrprError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class OpDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("nu", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("c", ctypes.c_double),
                ("dt", ctypes.c_double), ("bc", ctypes.c_int)]


class Panel(ctypes.Structure):
    _fields_ = [("F", ctypes.c_void_p), ("X", ctypes.c_void_p), ("ldx", ctypes.c_int64),
                ("w", ctypes.c_int), ("f", ctypes.c_void_p), ("ldf", ctypes.c_int64),
                ("fcol", ctypes.c_void_p), ("fscale", ctypes.c_void_p)]


class ServeOp(ctypes.Structure):
    _fields_ = [("C", ctypes.c_void_p), ("F", ctypes.POINTER(ctypes.c_void_p)), ("nsteps", ctypes.c_int),
                ("fscale", ctypes.c_void_p)]


class PararealProblem(ctypes.Structure):
    _fields_ = [("C", ctypes.c_void_p), ("F", ctypes.c_void_p), ("nreq", ctypes.c_int),
                ("u0", ctypes.c_void_p), ("f", ctypes.c_void_p), ("fscale", ctypes.c_void_p),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("U", ctypes.c_void_p),
                ("iters_host", ctypes.c_void_p), ("incr_host", ctypes.c_void_p), ("apost_host", ctypes.c_void_p)]


class SliceDesc(ctypes.Structure):
    _fields_ = [("F", ctypes.c_void_p), ("k", ctypes.c_int), ("p", ctypes.c_int),
                ("Omega", ctypes.c_void_p)]


_lib = None


def load():
    """Load liblrpr.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblrpr.so not built: run `python -m paper_2508_08873_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    lib.lrpr_ctx_create.argtypes = [i32, vp, P(vp)]
    lib.lrpr_ctx_destroy.argtypes = [vp]
    lib.lrpr_ctx_destroy.restype = None
    lib.lrpr_ctx_set_stream.argtypes = [vp, vp]
    lib.lrpr_last_error.argtypes = [vp]
    lib.lrpr_last_error.restype = ctypes.c_char_p
    lib.lrpr_factor.argtypes = [vp, P(OpDesc), i32, P(vp)]
    lib.lrpr_factor_stepper.argtypes = [vp, P(OpDesc), i32, i32, P(vp)]
    lib.lrpr_factor_sequence.argtypes = [vp, P(OpDesc), i32, i32, P(vp)]
    lib.lrpr_factor_many.argtypes = [vp, P(OpDesc), i32, i32, P(vp)]
    lib.lrpr_ctx_release_workspaces.argtypes = [vp]
    lib.lrpr_device_trim.argtypes = [i32]
    lib.lrpr_tune_set.argtypes = [vp, i32, i64]
    lib.lrpr_tune_get.argtypes = [vp, i32, P(i64)]
    lib.lrpr_autotune_factor.argtypes = [vp, P(OpDesc), i32, i32, P(i32), P(dbl)]
    lib.lrpr_factor_destroy.argtypes = [vp]
    lib.lrpr_factor_destroy.restype = None
    lib.lrpr_factor_info.argtypes = [vp, P(i64), P(i32), P(dbl)]
    lib.lrpr_factor_copy_lu.argtypes = [vp, vp, vp]
    lib.lrpr_factor_copy_tiles.argtypes = [vp, vp, i32, i32, vp]
    lib.lrpr_fine_step_batched.argtypes = [vp, i32, P(Panel), i32, i32]
    lib.lrpr_adjoint_step_batched.argtypes = [vp, i32, P(Panel), i32, i32]
    lib.lrpr_rsvd_build.argtypes = [vp, i32, P(SliceDesc), i32, i32, P(vp), vp, vp]
    lib.lrpr_rsvd_build_w.argtypes = [vp, i32, P(SliceDesc), vp, i32, i32, i32, P(vp), vp, vp]
    lib.lrpr_coarse_from_factors.argtypes = [vp, i32, vp, vp, vp, vp, vp, P(vp)]
    lib.lrpr_mass_weights.argtypes = [P(OpDesc), vp]
    lib.lrpr_coarse_destroy.argtypes = [vp]
    lib.lrpr_coarse_destroy.restype = None
    lib.lrpr_coarse_view.argtypes = [vp, i32, i32, P(vp)]
    lib.lrpr_coarse_get.argtypes = [vp, i32, P(vp), P(vp), P(vp), P(i32), P(i64)]
    lib.lrpr_coarse_apply.argtypes = [vp, vp, i32, i32, vp, vp]
    lib.lrpr_coarse_apply_noalloc.argtypes = [vp, vp, i32, i32, vp, vp]
    lib.lrpr_parareal_solve.argtypes = [vp, vp, P(vp), i32, i32, i32, vp, vp, vp, dbl, i32, vp, vp, vp, vp]
    lib.lrpr_parareal_solve_many.argtypes = [vp, i32, P(PararealProblem), i32, i32]
    lib.lrpr_profile_enable.argtypes = [vp, i32]
    lib.lrpr_profile_read.argtypes = [vp, P(dbl), P(i64), P(dbl), P(dbl), P(dbl)]
    lib.lrpr_randn.argtypes = [vp, vp, i64, i32, ctypes.c_uint64, ctypes.c_uint64]
    lib.lrpr_server_create.argtypes = [vp, i32, P(ServeOp), dbl, ctypes.c_size_t, i32, P(vp)]
    lib.lrpr_server_destroy.argtypes = [vp]
    lib.lrpr_server_destroy.restype = None
    lib.lrpr_server_submit.argtypes = [vp, i32, vp, vp, vp, P(i64)]
    lib.lrpr_server_progress.argtypes = [vp, i32, i32, P(i64), P(i32), P(i32)]
    lib.lrpr_server_stats.argtypes = [vp, P(i32), P(i32), P(i64)]
    lib.lrpr_server_last_error.argtypes = [vp]
    lib.lrpr_server_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("lrpr_ctx_destroy", "lrpr_factor_destroy", "lrpr_coarse_destroy", "lrpr_last_error",
                        "lrpr_server_destroy", "lrpr_server_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _opdesc(dim, nx, nu, beta, c, dt, bc=BC_DIRICHLET):
    return OpDesc(dim, nx, float(nu), float(beta[0]), float(beta[1]) if dim == 2 else 0.0, float(c), float(dt),
                  int(bc))


def mass_weights(dim, nx, bc=BC_DIRICHLET):
    """Lumped-mass weights of the grid (lrpr_mass_weights, host), as a NumPy array."""
    import numpy as np
    lib = load()
    n = nx if dim == 1 else nx * nx
    w = np.zeros(n, dtype=np.float64)
    d = _opdesc(dim, nx, 1.0, (0.0, 0.0), 0.0, 1.0, bc)
    st = lib.lrpr_mass_weights(ctypes.byref(d), w.ctypes.data_as(ctypes.c_void_p))
    if st != 0:
        raise LrprError(st, "lrpr_mass_weights")
    return w


class Context:
    """lrpr_ctx bound to a torch device; uses torch's current stream."""

    def __init__(self, device: int = 0):
        self.lib = load()
        self.device = device
        h = ctypes.c_void_p()
        stream = torch.cuda.current_stream(device).cuda_stream
        self._check(self.lib.lrpr_ctx_create(device, ctypes.c_void_p(stream), ctypes.byref(h)), ctx=None)
        self.h = h

    def _check(self, st, ctx="self"):
        if st != 0:
            msg = ""
            if ctx == "self":
                msg = self.lib.lrpr_last_error(self.h).decode()
            raise LrprError(st, msg)

    def sync_stream(self):
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self.lib.lrpr_ctx_set_stream(self.h, ctypes.c_void_p(stream))

    def close(self):
        if getattr(self, "h", None):
            self.lib.lrpr_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- sweep timing -----------------------------------------------------
    def profile(self, enable=True):
        self._check(self.lib.lrpr_profile_enable(self.h, int(enable)))

    def profile_read(self):
        ms, fl, by, rs = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        nl = ctypes.c_int64()
        self._check(self.lib.lrpr_profile_read(self.h, ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(fl),
                                               ctypes.byref(by), ctypes.byref(rs)))
        return {"ms": ms.value, "launches": nl.value, "flops": fl.value, "bytes": by.value, "rhs_steps": rs.value}

    # -- random test matrices ---------------------------------------------
    def randn(self, X, seed, stream):
        """Fill the contiguous float64/float32 cuda tensor X with the library's
        Philox4x32-10 + Box-Muller Gaussians of (seed, stream)."""
        prec = LRPR_F64 if X.dtype == torch.float64 else LRPR_F32
        self.sync_stream()
        self._check(self.lib.lrpr_randn(self.h, ctypes.c_void_p(X.data_ptr()), ctypes.c_int64(X.numel()), int(prec),
                                        ctypes.c_uint64(seed), ctypes.c_uint64(stream)))
        return X

    # -- factor -----------------------------------------------------------
    def factor(self, dim, nx, nu, beta, c, dt, store_mask=1, stepper=STEP_EULER, bc=BC_DIRICHLET):
        d = _opdesc(dim, nx, nu, beta, c, dt, bc)
        h = ctypes.c_void_p()
        self.sync_stream()
        if stepper == STEP_EULER:
            self._check(self.lib.lrpr_factor(self.h, ctypes.byref(d), int(store_mask), ctypes.byref(h)))
        else:
            self._check(self.lib.lrpr_factor_stepper(self.h, ctypes.byref(d), int(store_mask), int(stepper),
                                                     ctypes.byref(h)))
        return Factor(self, h)

    def factor_sequence(self, ops, store_mask=1):
        """Per-step operators: ops is a list of dicts (dim, nx, nu, beta, c, dt),
        one per implicit-Euler step (lrpr_factor_sequence)."""
        arr = (OpDesc * len(ops))()
        for j, o in enumerate(ops):
            b = o["beta"]
            arr[j] = _opdesc(o["dim"], o["nx"], o["nu"], b, o["c"], o["dt"], o.get("bc", BC_DIRICHLET))
        h = ctypes.c_void_p()
        self.sync_stream()
        self._check(self.lib.lrpr_factor_sequence(self.h, arr, len(ops), int(store_mask), ctypes.byref(h)))
        return Factor(self, h)

    def factor_many(self, ops, store_mask=1):
        """Independent factors of operators on one grid (lrpr_factor_many):
        ops is a list of dicts (dim, nx, nu, beta, c, dt); returns Factors."""
        arr = (OpDesc * len(ops))()
        for j, o in enumerate(ops):
            arr[j] = _opdesc(o["dim"], o["nx"], o["nu"], o["beta"], o["c"], o["dt"], o.get("bc", BC_DIRICHLET))
        hs = (ctypes.c_void_p * len(ops))()
        self.sync_stream()
        self._check(self.lib.lrpr_factor_many(self.h, arr, len(ops), int(store_mask), hs))
        return [Factor(self, ctypes.c_void_p(hs[j])) for j in range(len(ops))]

    def tune_set(self, param, value):
        self._check(self.lib.lrpr_tune_set(self.h, int(param), int(value)))

    def tune_get(self, param):
        v = ctypes.c_int64()
        self._check(self.lib.lrpr_tune_get(self.h, int(param), ctypes.byref(v)))
        return v.value

    def autotune_factor(self, dim, nx, nu, beta, c, dt, count, store_mask=1):
        """lrpr_autotune_factor: returns (workgroups per matrix, ms)."""
        d = _opdesc(dim, nx, nu, beta, c, dt)
        wg, ms = ctypes.c_int(), ctypes.c_double()
        self.sync_stream()
        self._check(self.lib.lrpr_autotune_factor(self.h, ctypes.byref(d), int(count), int(store_mask),
                                                  ctypes.byref(wg), ctypes.byref(ms)))
        return wg.value, ms.value

    def parareal_solve_many(self, problems, nsteps, fine_prec=LRPR_F64):
        return _parareal_many(self, problems, nsteps, fine_prec)

    def device_trim(self):
        self._check(self.lib.lrpr_device_trim(self.device))

    def release_workspaces(self):
        self.sync_stream()
        self._check(self.lib.lrpr_ctx_release_workspaces(self.h))

    # -- sweeps -----------------------------------------------------------
    def _panels(self, specs):
        arr = (Panel * len(specs))()
        for i, s in enumerate(specs):
            X = s["X"]
            f = s.get("f")
            arr[i] = Panel(s["F"].h, X.data_ptr(), X.stride(1) if X.dim() == 2 and X.shape[1] > 1 else X.shape[0],
                           X.shape[1] if X.dim() == 2 else 1,
                           f.data_ptr() if f is not None else None,
                           (f.stride(1) if f.dim() == 2 and f.shape[1] > 1 else f.shape[0]) if f is not None else 0,
                           s["fcol"].data_ptr() if s.get("fcol") is not None else None,
                           s["fscale"].data_ptr() if s.get("fscale") is not None else None)
        return arr

    def fine_step_batched(self, specs, nsteps, prec=LRPR_F64):
        """specs: list of dicts {F, X (n x w, column-major = t().contiguous().t()), f, fcol, fscale}."""
        arr = self._panels(specs)
        self.sync_stream()
        self._check(self.lib.lrpr_fine_step_batched(self.h, len(specs), arr, int(nsteps), int(prec)))

    def adjoint_step_batched(self, specs, nsteps, prec=LRPR_F64):
        arr = self._panels(specs)
        self.sync_stream()
        self._check(self.lib.lrpr_adjoint_step_batched(self.h, len(specs), arr, int(nsteps), int(prec)))

    # -- rSVD -------------------------------------------------------------
    def rsvd_build(self, slices, nsteps, range_prec=LRPR_F64, q=0, psi=None, weights=None):
        """slices: list of (Factor, k, p, Omega tensor n x (k+p) column-major);
        q power iterations (lrpr_rsvd_build_q); psi: per-slice independent
        adjoint test matrices (lrpr_rsvd_build_two_sided); weights: per-slice
        float64 cuda tensors of n inner-product weights, or None entries
        (lrpr_rsvd_build_w)."""
        arr = (SliceDesc * len(slices))()
        tot = 0
        for i, (F, k, p, Om) in enumerate(slices):
            arr[i] = SliceDesc(F.h, int(k), int(p), Om.data_ptr() if Om is not None else None)
            tot += k + p
        sig = (ctypes.c_double * max(tot, 1))()
        fb = (ctypes.c_int * max(len(slices), 1))()
        h = ctypes.c_void_p()
        self.sync_stream()
        if weights is not None:
            ww = (ctypes.c_void_p * len(slices))(*[t.data_ptr() if t is not None else None for t in weights])
            self._check(self.lib.lrpr_rsvd_build_w(self.h, len(slices), arr, ww, int(nsteps), int(q),
                                                   int(range_prec), ctypes.byref(h), sig, fb))
        elif psi is not None:
            pp = (ctypes.c_void_p * len(slices))(*[t.data_ptr() for t in psi])
            self._check(self.lib.lrpr_rsvd_build_two_sided(self.h, len(slices), arr, pp, int(nsteps),
                                                           int(range_prec), ctypes.byref(h), sig, fb))
        elif q:
            self._check(self.lib.lrpr_rsvd_build_q(self.h, len(slices), arr, int(nsteps), int(q), int(range_prec),
                                                   ctypes.byref(h), sig, fb))
        else:
            self._check(self.lib.lrpr_rsvd_build(self.h, len(slices), arr, int(nsteps), int(range_prec),
                                                 ctypes.byref(h), sig, fb))
        return Coarse(self, h, [F for (F, _, _, _) in slices], list(sig)[:tot], list(fb)[:len(slices)],
                      ls=[k + p for (_, k, p, _) in slices])

    def coarse_from_factors(self, factors, U, S, V):
        """A priori coarse solvers (lrpr_coarse_from_factors): per slice float64
        cuda tensors U (n x k column-major), S (k,), V (n x k column-major)."""
        N = len(factors)
        fa = (ctypes.c_void_p * N)(*[F.h.value for F in factors])
        ks = (ctypes.c_int * N)(*[int(u.shape[1]) for u in U])
        up = (ctypes.c_void_p * N)(*[u.data_ptr() for u in U])
        sp = (ctypes.c_void_p * N)(*[x.data_ptr() for x in S])
        vp = (ctypes.c_void_p * N)(*[v.data_ptr() for v in V])
        h = ctypes.c_void_p()
        self.sync_stream()
        self._check(self.lib.lrpr_coarse_from_factors(self.h, N, fa, ks, up, sp, vp, ctypes.byref(h)))
        sig = []
        for x in S:
            sig += [float(v) for v in x.cpu()]
        return Coarse(self, h, list(factors), sig, [0] * N)

    # -- Parareal ---------------------------------------------------------
    def parareal_solve(self, coarse, factors, nsteps, u0, f=None, fscale=None, tol=1e-10, max_iter=None,
                       fine_prec=LRPR_F64):
        """u0: (n, nreq) float64 cuda column-major; f: (n, nreq) or None; fscale: (N*nsteps,) float64."""
        N = len(factors)
        if max_iter is None:
            max_iter = N
        n, nreq = u0.shape
        U = torch.zeros((nreq, N + 1, n), dtype=torch.float64, device=u0.device)
        fa = (ctypes.c_void_p * N)(*[F.h.value for F in factors])
        iters = (ctypes.c_int * nreq)()
        incr = (ctypes.c_double * (nreq * max_iter))()
        apost = (ctypes.c_double * (nreq * N))()
        self.sync_stream()
        st = self.lib.lrpr_parareal_solve(self.h, coarse.h, fa, int(nsteps), int(fine_prec), int(nreq),
                                          _ptr(u0), _ptr(f), _ptr(fscale), float(tol), int(max_iter),
                                          _ptr(U), iters, incr, apost)
        if st not in (0, 5):
            self._check(st)
        return {"U": U, "iters": list(iters), "incr": [list(incr[r * max_iter:(r + 1) * max_iter]) for r in range(nreq)],
                "apost": [list(apost[r * N:(r + 1) * N]) for r in range(nreq)], "status": st}


def _parareal_many(ctx, problems, nsteps, fine_prec):
    """lrpr_parareal_solve_many; problems: list of dicts {coarse, factors,
    u0 (n x nreq), f or None, fscale or None, tol, max_iter or None}."""
    arr = (PararealProblem * len(problems))()
    keep, outs = [], []
    for i, pr in enumerate(problems):
        facs = pr["factors"]
        N = len(facs)
        mi = pr.get("max_iter") or N
        u0 = pr["u0"]
        n, nreq = u0.shape
        U = torch.zeros((nreq, N + 1, n), dtype=torch.float64, device=u0.device)
        fa = (ctypes.c_void_p * N)(*[F.h.value for F in facs])
        iters = (ctypes.c_int * nreq)()
        incr = (ctypes.c_double * (nreq * mi))()
        apost = (ctypes.c_double * (nreq * N))()
        keep += [fa, iters, incr, apost, U]
        addr = lambda t: t.data_ptr() if t is not None else None
        arr[i] = PararealProblem(pr["coarse"].h, ctypes.cast(fa, ctypes.c_void_p), nreq, addr(u0), addr(pr.get("f")),
                                 addr(pr.get("fscale")), float(pr["tol"]), int(mi), addr(U),
                                 ctypes.cast(iters, ctypes.c_void_p), ctypes.cast(incr, ctypes.c_void_p),
                                 ctypes.cast(apost, ctypes.c_void_p))
        outs.append((U, iters, incr, apost, nreq, mi, N))
    ctx.sync_stream()
    st = ctx.lib.lrpr_parareal_solve_many(ctx.h, len(problems), arr, int(nsteps), int(fine_prec))
    if st not in (0, 5):
        ctx._check(st)
    res = []
    for U, iters, incr, apost, nreq, mi, N in outs:
        res.append({"U": U, "iters": list(iters), "incr": [list(incr[r * mi:(r + 1) * mi]) for r in range(nreq)],
                    "apost": [list(apost[r * N:(r + 1) * N]) for r in range(nreq)], "status": st})
    return res


class Factor:
    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h
        n, bw, dt = ctypes.c_int64(), ctypes.c_int(), ctypes.c_double()
        ctx.lib.lrpr_factor_info(h, ctypes.byref(n), ctypes.byref(bw), ctypes.byref(dt))
        self.n, self.bw, self.dt = n.value, bw.value, dt.value

    def lu_host(self):
        import numpy as np
        out = np.zeros((self.n, 2 * self.bw + 1), dtype=np.float64)
        self.ctx._check(self.ctx.lib.lrpr_factor_copy_lu(self.ctx.h, self.h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def tiles_host(self, which, prec):
        """Packed band tiles (which: 0 lower, 1 upper; prec LRPR_F64 or
        LRPR_F32) as an array [NT, nb, 256] in the tiles' own element order."""
        import numpy as np
        NT, nb = (self.n + 15) // 16, (self.bw + 15) // 16
        out = np.zeros((NT, nb, 256), dtype=np.float32 if prec == LRPR_F32 else np.float64)
        self.ctx._check(self.ctx.lib.lrpr_factor_copy_tiles(self.ctx.h, self.h, which, prec,
                                                            out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.lrpr_factor_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Coarse:
    def __init__(self, ctx, h, factors, sigma, fallback, parent=None, ls=None):
        self.ctx, self.h, self.factors, self.sigma, self.fallback = ctx, h, factors, sigma, fallback
        self.parent = parent   # a view keeps the handle it shares memory with alive
        self.ls = ls           # singular values per slice (sigma is their concatenation)

    def get(self, s):
        """(U, S, V) of slice s copied into new torch tensors (n x k, k+p, n x k)."""
        U, S, V = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        k, n = ctypes.c_int(), ctypes.c_int64()
        self.ctx._check(self.ctx.lib.lrpr_coarse_get(self.h, s, ctypes.byref(U), ctypes.byref(S), ctypes.byref(V),
                                                     ctypes.byref(k), ctypes.byref(n)))
        return k.value, n.value, U.value, S.value, V.value

    def view(self, first, count):
        """lrpr_coarse_view: slices [first, first+count) as a handle of their
        own (no device memory of its own; this handle must outlive it)."""
        h = ctypes.c_void_p()
        self.ctx._check(self.ctx.lib.lrpr_coarse_view(self.h, int(first), int(count), ctypes.byref(h)))
        ls = self.ls[first:first + count] if self.ls else None
        pos = sum(self.ls[:first]) if self.ls else 0
        sig = self.sigma[pos:pos + sum(ls)] if ls else []
        return Coarse(self.ctx, h, self.factors[first:first + count] if self.factors else self.factors,
                      sig, self.fallback[first:first + count] if self.fallback else self.fallback, parent=self, ls=ls)

    def apply(self, s, Vin):
        out = torch.empty_like(Vin)
        self.ctx.sync_stream()
        self.ctx._check(self.ctx.lib.lrpr_coarse_apply(self.ctx.h, self.h, s, Vin.shape[1], _ptr(Vin), _ptr(out)))
        return out

    def apply_noalloc(self, s, Vin, out=None):
        """lrpr_coarse_apply_noalloc into out (allocated here if None)."""
        if out is None:
            out = torch.empty_like(Vin)
        self.ctx.sync_stream()
        self.ctx._check(self.ctx.lib.lrpr_coarse_apply_noalloc(self.ctx.h, self.h, s, Vin.shape[1], _ptr(Vin),
                                                               _ptr(out)))
        return out

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.lrpr_coarse_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """lrpr_server: continuous batching of Parareal solves over device-resident
    coarse propagators.  ops: list of (coarse, factors (list of N), nsteps,
    fscale tensor (N*nsteps doubles) or None)."""

    def __init__(self, ctx, ops, tol, budget_bytes, max_active=0):
        self.ctx, self.lib = ctx, ctx.lib
        self._keep = []
        arr = (ServeOp * len(ops))()
        self.n, self.N = [], []
        for i, (coarse, facs, nsteps, fsc) in enumerate(ops):
            fa = (ctypes.c_void_p * len(facs))(*[f.h.value for f in facs])
            self._keep += [coarse, facs, fa, fsc]
            arr[i] = ServeOp(coarse.h, ctypes.cast(fa, ctypes.POINTER(ctypes.c_void_p)), int(nsteps),
                             fsc.data_ptr() if fsc is not None else None)
            self.n.append(facs[0].n)
            self.N.append(len(facs))
        h = ctypes.c_void_p()
        ctx.sync_stream()
        torch.cuda.current_stream(ctx.device).synchronize()
        ctx._check(self.lib.lrpr_server_create(ctx.h, len(ops), arr, float(tol), int(budget_bytes), int(max_active),
                                               ctypes.byref(h)))
        self.h = h
        self.pending = {}

    def _check(self, st):
        if st != 0:
            raise LrprError(st, self.lib.lrpr_server_last_error(self.h).decode())

    def submit(self, op, u0, f, sync=True):
        """Queue a request; returns (id, U) with U the n x (N+1) output
        (column-major, filled when the request is reported done)."""
        if sync:
            torch.cuda.current_stream(self.ctx.device).synchronize()
        n, N = self.n[op], self.N[op]
        U = torch.empty((N + 1, n), dtype=torch.float64, device=u0.device).t()
        rid = ctypes.c_int64()
        self._check(self.lib.lrpr_server_submit(self.h, int(op), _ptr(u0), _ptr(f), _ptr(U), ctypes.byref(rid)))
        self.pending[rid.value] = (u0, f, U)
        return rid.value, U

    def progress(self, wait=True, max_done=4096):
        """Advance the server; returns [(id, iterations)] of requests done."""
        ids = (ctypes.c_int64 * max_done)()
        its = (ctypes.c_int * max_done)()
        nd = ctypes.c_int()
        self._check(self.lib.lrpr_server_progress(self.h, 1 if wait else 0, max_done, ids, its, ctypes.byref(nd)))
        out = []
        for i in range(nd.value):
            self.pending.pop(ids[i], None)
            out.append((ids[i], its[i]))
        return out

    def stats(self):
        q, a, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
        self._check(self.lib.lrpr_server_stats(self.h, ctypes.byref(q), ctypes.byref(a), ctypes.byref(b)))
        return {"queued": q.value, "active": a.value, "bytes_in_use": b.value}

    def close(self):
        if getattr(self, "h", None):
            self.lib.lrpr_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DevArray:
    """Exposes a library-owned device array through __cuda_array_interface__."""

    def __init__(self, ptr, shape, typestr):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (int(ptr), False),
                                         "version": 2, "strides": None}


def device_view(ptr, n, k, dtype=torch.float64):
    """Column-major n x k device array at ptr (library-owned), as a torch
    tensor view (no copy; valid while the owning handle lives)."""
    ts = {torch.float64: "<f8", torch.float32: "<f4"}[dtype]
    t = torch.as_tensor(_DevArray(ptr, (k, n), ts), device="cuda")
    return t.t()


def colmajor(t):
    """Column-major (Fortran-order) copy of a 2-D tensor: element (i, c) at i + c*n."""
    return t.t().contiguous().t()
