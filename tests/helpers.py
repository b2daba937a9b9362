"""Shared test helpers: conversions between the oracle's sparse matrices and
the library's 9-plane stencil layout (plane p = (di+1) + 3 (dj+1))."""
import numpy as np


def planes_from_csr(A, N):
    s = N + 1
    n = s * s
    out = np.zeros((9, n))
    coo = A.tocoo()
    r, c, v = coo.row, coo.col, coo.data
    di = (c % s) - (r % s)
    dj = (c // s) - (r // s)
    assert np.all(np.abs(di) <= 1) and np.all(np.abs(dj) <= 1)
    p = (di + 1) + 3 * (dj + 1)
    np.add.at(out, (p, r), v)
    return out


def rel_max(a, b):
    scale = max(np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() / scale
