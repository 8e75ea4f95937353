"""Row-sum-keeping FP32 rounding of packed factor rows, as the library's
header states the rule: every entry of a row is rounded to FP32; the FP64
sum of the rounding errors is added to the largest entry (by magnitude,
first one on ties); what the rounding of that entry leaves is added to the
smallest entry of at least 2^-12 of the largest (strictly smaller than the
largest, not the largest itself, first one on ties).  Test infrastructure:
two independent writings of the rule, one literal, one over whole arrays."""
import numpy as np


def rule_row_literal(v):
    """One row, entry by entry (plain Python floats are FP64)."""
    v = [float(x) for x in v]
    f = [float(np.float32(x)) for x in v]
    err = 0.0
    vmax, at = 0.0, -1
    for t, x in enumerate(v):
        err += x - f[t]
        if abs(x) > abs(vmax):
            vmax, at = x, t
    out = np.array(f, dtype=np.float32)
    if at < 0:
        return out
    want = f[at] + err
    out[at] = np.float32(want)
    res = want - float(out[at])
    if res == 0.0:
        return out
    lo = abs(vmax) / 4096.0
    best, at2 = abs(vmax), -1
    for t, x in enumerate(v):
        if t != at and abs(x) >= lo and abs(x) < best:
            best, at2 = abs(x), t
    if at2 >= 0:
        out[at2] = np.float32(float(out[at2]) + res)
    return out


def rule_rows(V):
    """Every row of V (FP64, [rows, entries]) at once."""
    F = V.astype(np.float32)
    err = (V - F.astype(np.float64)).sum(axis=1)
    A = np.abs(V)
    amax = A.max(axis=1)
    imax = A.argmax(axis=1)
    rows = np.arange(V.shape[0])
    ok = amax > 0
    want = F[rows, imax].astype(np.float64) + err
    fat = want.astype(np.float32)
    res = want - fat.astype(np.float64)
    cols = np.arange(V.shape[1]).reshape(1, -1)
    mask = (A >= (amax / 4096.0).reshape(-1, 1)) & (A < amax.reshape(-1, 1)) & (cols != imax.reshape(-1, 1))
    at2 = np.where(mask, A, np.inf).argmin(axis=1)
    ok2 = ok & (res != 0) & mask.any(axis=1)
    F[rows[ok], imax[ok]] = fat[ok]
    F[rows[ok2], at2[ok2]] = (F[rows[ok2], at2[ok2]].astype(np.float64) + res[ok2]).astype(np.float32)
    return F
