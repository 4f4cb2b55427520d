"""Test helper: the matrix of the oracle's apply_h, recovered by probing.

A column (l, i) of H touches rows (l, i +- k) for k <= s and (l +- 1, i) (the
velocity gauge: (l +- 1, i +- k) as well).  Two columns with equal l mod 3 and
equal i mod (2s+1) never touch a common row, so 3(2s+1) probe vectors recover
every entry of H.
"""
import numpy as np
import scipy.sparse as sp


def sparse_h(orc, g, efield):
    s = 1 if g.stencil == 3 else 2
    w = 2 * s + 1
    n, nl = g.n, g.lmax + 1
    li = np.repeat(np.arange(nl), n)
    ii = np.tile(np.arange(n), nl)
    color = (li % 3) * w + (ii % w)
    rows, cols, vals = [], [], []
    for c in range(3 * w):
        probe = (color == c).astype(np.complex128)
        out = orc.apply_h(g, efield, probe)
        for dl in (-1, 0, 1):
            for di in range(-s, s + 1):
                # the length gauge couples rows l +- 1 at the same radius only;
                # the velocity gauge through the radial derivative as well
                if dl != 0 and di != 0 and getattr(g, "gauge", 0) == 0:
                    continue
                # rows r = (l+dl, i+di) of the probed columns (l, i)
                col = np.nonzero(probe)[0]
                l = li[col] + dl
                i = ii[col] + di
                ok = (l >= 0) & (l < nl) & (i >= 0) & (i < n)
                r = l[ok] * n + i[ok]
                rows.append(r)
                cols.append(col[ok])
                vals.append(out[r])
    m = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(g.size, g.size))
    return m
