"""Host-side checks of the C-ABI boundary and of the benchmark's contract.

* every function include/lrpr.h declares is exported by liblrpr.so, and the
  Python binding names the same set;
* the C structs mirrored in the binding have the sizes the header implies;
* argument errors are reported without touching a device (null context);
* ``bench.py --gpus 2`` refuses to run (one GPU only).
"""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lrpr.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(lrpr_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2508_08873_amd import build, lrpr
    if not os.path.exists(lrpr.LIB_PATH):
        build.build()
    return lrpr.load()


def test_header_declares_the_paths_entry_points():
    names = _declared()
    for fn in ["lrpr_factor", "lrpr_fine_step_batched", "lrpr_adjoint_step_batched", "lrpr_rsvd_build",
               "lrpr_parareal_solve"]:
        assert fn in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_declared_symbol():
    from paper_2508_08873_amd import lrpr
    assert sorted(lrpr.EXPORTS) == _declared()


def test_struct_layouts():
    from paper_2508_08873_amd import lrpr
    # lrpr_op_desc: int, int, 5 doubles, int (+pad)
    assert ctypes.sizeof(lrpr.OpDesc) == 8 + 5 * 8 + 8
    # lrpr_panel: F, X, ldx, w(+pad), f, ldf, fcol, fscale
    assert ctypes.sizeof(lrpr.Panel) == 8 * 8
    # lrpr_slice_desc: F, k, p, Omega
    assert ctypes.sizeof(lrpr.SliceDesc) == 8 + 4 + 4 + 8
    # lrpr_parareal_problem: C, F, nreq(+pad), u0, f, fscale, tol, max_iter(+pad), U, iters, incr, apost
    assert ctypes.sizeof(lrpr.PararealProblem) == 12 * 8
    assert lrpr.PararealProblem.tol.offset == 48 and lrpr.PararealProblem.U.offset == 64


def test_mass_weights_host_entry_point(ora):
    """lrpr_mass_weights is host code: against the oracle's lumped mass."""
    from paper_2508_08873_amd import lrpr
    for dim, nx, bc, name in ((1, 7, 1, "neumann"), (2, 5, 1, "neumann"), (1, 6, 0, "dirichlet"), (2, 3, 0, "dirichlet")):
        assert np.array_equal(lrpr.mass_weights(dim, nx, bc), ora.mass_weights(dim, nx, name))
    with pytest.raises(lrpr.LrprError):
        lrpr.mass_weights(1, 1, lrpr.BC_NEUMANN)


def test_null_context_is_an_argument_error(lib):
    # no device is touched: every entry point validates its handle first
    assert lib.lrpr_factor(None, None, 1, None) == 1
    assert lib.lrpr_fine_step_batched(None, 0, None, 1, 0) == 1
    assert lib.lrpr_adjoint_step_batched(None, 0, None, 1, 0) == 1
    assert lib.lrpr_parareal_solve_many(None, 1, None, 1, 0) == 1
    assert lib.lrpr_tune_set(None, 1, 0) == 1
    assert lib.lrpr_factor_many(None, None, 1, 1, None) == 1
    assert lib.lrpr_last_error(None) == b"null context"


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
