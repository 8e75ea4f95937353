"""The packed band tiles that every sweep reads, checked directly.

FP64 tiles: L(I,I)^{-1} L(I, I-nb+j) and U(I,I)^{-1} U(I, I+1+j) of the
factor's own band LU (Sec. 4.4: the factorisation that every solve reuses),
formed here with numpy's inverse and products from the copied band: within
1e-12 of each tile row's largest entry.

FP32 tiles: the row-sum-keeping rounding of the FP64 tiles, applied here to
the FP64 tiles the library keeps, entry by entry as the header states it
(every entry rounded; the FP64 sum of the rounding errors into the largest
entry; what that leaves into the smallest entry of at least 2^-12 of the
largest; ties to the first entry).  Bit for bit: the library sums the
errors in another order, which moves the FP32 results only if a sum lands
within about 1e-16 of its size from a rounding boundary.
"""
import numpy as np
import pytest
from packrule import rule_rows

from paper_2508_08873_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2508_08873_amd import lrpr
    return lrpr.Context(0)


def _pos():
    r = np.arange(16).reshape(16, 1)
    k = np.arange(16).reshape(1, 16)
    p64 = 128 * (k // 8) + 2 * (16 * (k % 4) + r) + (k // 4) % 2
    p32 = 4 * (16 * (k // 4) + r) + k % 4
    return p64, p32


def _rows(T, pos, I):
    """Rows of tile rows I: [len(I) * 16, 16 nb] with entry (j, k) at 16 j + k."""
    nb = T.shape[1]
    sub = T[I]                                   # [nI, nb, 256]
    out = sub[:, :, pos]                         # [nI, nb, 16 (r), 16 (k)]
    return out.transpose(0, 2, 1, 3).reshape(len(I) * 16, nb * 16)


def _block(lu, n, bw, I, J, upper):
    """Dense 16x16 blocks (I[t], J[t]) of the unit-lower L (upper=False) or of
    U (upper=True) from the band storage; rows past n are identity rows."""
    out = np.zeros((len(I), 16, 16))
    for r in range(16):
        i = 16 * I + r
        for k in range(16):
            c = 16 * J + k
            inb = (i < n) & (c >= 0) & (c < n) & (np.abs(c - i) <= bw)
            tri = (c >= i) if upper else (c < i)
            take = inb & tri
            v = np.zeros(len(I))
            v[take] = lu[i[take], (c - i + bw)[take]]
            diag = c == i
            if not upper:
                v[diag] = 1.0
            else:
                v[diag & (i >= n)] = 1.0
            out[:, r, k] = v
    return out


CASES = [("heat1d", dict()), ("nx100", dict(nx=100)), ("nx300", dict(nx=300, beta=(-6.0, 14.0))),
         ("nx520", dict(nx=520))]


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_packed_tiles(ctx, name, kw):
    from paper_2508_08873_amd import lrpr
    P = inputs.heat1d(**kw) if name == "heat1d" else inputs.tiny2d(**kw)
    F = ctx.factor(P.dim, P.nx, P.nu, P.beta, P.c, P.dt, store_mask=lrpr.STORE_F64 | lrpr.STORE_F32)
    n, bw = F.n, F.bw
    NT, nb = (n + 15) // 16, (bw + 15) // 16
    lu = F.lu_host()
    p64, p32 = _pos()
    # every tile row for small factors, a spread sample (first, last, interior) for large ones
    I = np.arange(NT) if NT <= 700 else np.unique(np.concatenate([np.arange(3), np.arange(NT - 3, NT),
                                                                     np.linspace(0, NT - 1, 400).astype(int)]))
    for which in (0, 1):
        print(name, "n", n, "nb", nb, "set", which, "tile rows", len(I), flush=True)
        T64 = F.tiles_host(which, lrpr.LRPR_F64)
        T32 = F.tiles_host(which, lrpr.LRPR_F32)
        # FP64 tiles against numpy's products of the copied LU
        D = np.linalg.inv(_block(lu, n, bw, I, I, upper=bool(which)))
        refs, gots = [], []
        for j in range(nb):
            J = I - nb + j if which == 0 else I + 1 + j
            refs.append(D @ _block(lu, n, bw, I, J, upper=bool(which)))
            gots.append(T64[I, j][:, p64])
            outside = (J < 0) | (J >= NT)
            assert not np.any(gots[-1][outside]), (which, j)
        ref, got = np.stack(refs, axis=1), np.stack(gots, axis=1)     # [nI, nb, 16, 16]
        scale = np.abs(ref).reshape(len(I), -1).max(axis=1).reshape(-1, 1, 1, 1)
        worst = float(np.max(np.abs(got - ref) / np.maximum(scale, 1e-300)))
        print("  FP64 tiles: worst entry error / tile-row max", worst, flush=True)
        assert worst <= 1e-12
        # FP32 tiles: the rounding rule on the library's own FP64 tiles
        V = _rows(T64, p64, I)
        G = _rows(T32, p32, I)
        E = rule_rows(V)
        bad = np.nonzero(E.view(np.uint32) != G.view(np.uint32))
        print("  FP32 tiles: entries differing from the rule", len(bad[0]), "of", E.size, flush=True)
        assert len(bad[0]) == 0, (bad[0][:5], bad[1][:5])
        # and the row sums kept: to within one rounding of the entry that
        # takes the last residual (at most the largest entry)
        ds = np.abs(G.astype(np.float64).sum(axis=1) - V.sum(axis=1))
        rs = np.abs(V).max(axis=1)
        assert np.all(ds <= 2.0 ** -24 * rs), float((ds / np.maximum(rs, 1e-300)).max())
    F.close()
