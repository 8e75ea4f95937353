"""The array form of the FP32 row rounding rule (used by the GPU test of the
packed tiles) against the rule written entry by entry, on rows with ties of
the largest and of the smallest entries, zeros, all-zero rows, entries below
2^-12 of the largest, and rows whose rounding errors cancel exactly."""
import numpy as np

from packrule import rule_row_literal, rule_rows


def _cases():
    r = np.random.default_rng(5)
    rows = [r.standard_normal(48) * np.exp(r.uniform(-8, 2, 48)) for _ in range(200)]
    t = r.standard_normal(32)
    t[[3, 17]] = 5.0                       # tie of the largest
    t[[5, 9, 30]] = 0.25 + 2.0 ** -30      # tie of the smallest candidate
    rows.append(t)
    rows.append(np.zeros(32))
    z = np.zeros(32)
    z[7] = -1.0 / 3.0                      # one nonzero entry
    rows.append(z)
    w = np.full(32, 1e-6)
    w[0] = 1.0 + 2.0 ** -40                # the others below 2^-12 of the largest
    rows.append(w)
    rows.append(np.full(32, 0.5))          # exactly representable: no residual
    rows.append(np.array([1.0 / 3.0, -1.0 / 3.0] * 16))
    return rows


def test_array_rule_equals_literal_rule():
    for v in _cases():
        want = rule_row_literal(v)
        got = rule_rows(np.asarray(v, dtype=np.float64).reshape(1, -1))[0]
        assert np.array_equal(want.view(np.uint32), got.view(np.uint32)), v


def test_rule_keeps_row_sums_better_than_plain_rounding():
    r = np.random.default_rng(9)
    V = r.standard_normal((400, 64)) * np.exp(r.uniform(-4, 0, (400, 64)))
    plain = np.abs(V.astype(np.float32).astype(np.float64).sum(axis=1) - V.sum(axis=1))
    kept = np.abs(rule_rows(V).astype(np.float64).sum(axis=1) - V.sum(axis=1))
    assert np.median(kept) < 1e-3 * np.median(plain)
    assert np.all(kept <= 2.0 ** -24 * np.abs(V).max(axis=1))
