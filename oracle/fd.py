"""Finite-difference weights and 1-D difference matrices (test infrastructure, see package header).

The paper discretises with high-order finite differences in a method-of-lines setting (Sec. 3)
and runs its experiments with sixth-order operators (Sec. 5.2). First derivatives use
seven-point windows: centred where the nodes exist, shifted to stay inside the node range
otherwise (ghost nodes included). Weights come from Fornberg's recursion (Fornberg 1988,
"Generation of finite difference formulas on arbitrarily spaced grids").

Pins (tests/test_oracle_fd.py): the centred sixth-order first-derivative weights
(-1/60, 3/20, -3/4, 0, 3/4, -3/20, 1/60)/h, exactness on monomials of degree <= window-1 for
every shifted window, rows summing to zero, the 3-point second-derivative (1, -2, 1)/h^2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def fornberg(z: float, nodes, mmax: int) -> np.ndarray:
    """Weights c[i, m] such that sum_i c[i, m] f(nodes[i]) ~ f^(m)(z), m = 0..mmax."""
    x = np.asarray(nodes, dtype=np.float64)
    n = x.size
    c = np.zeros((n, mmax + 1))
    c1 = 1.0
    c4 = x[0] - z
    c[0, 0] = 1.0
    for i in range(1, n):
        mn = min(i, mmax)
        c2 = 1.0
        c5 = c4
        c4 = x[i] - z
        for j in range(i):
            c3 = x[i] - x[j]
            c2 *= c3
            if j == i - 1:
                for k in range(mn, 0, -1):
                    c[i, k] = c1 * (k * c[i - 1, k - 1] - c5 * c[i - 1, k]) / c2
                c[i, 0] = -c1 * c5 * c[i - 1, 0] / c2
            for k in range(mn, 0, -1):
                c[j, k] = (c4 * c[j, k] - k * c[j, k - 1]) / c3
            c[j, 0] = c4 * c[j, 0] / c3
        c1 = c2
    return c


def window_start(i: int, npts: int, width: int) -> int:
    """First node of the width-point window used at node i of a non-periodic line."""
    hw = width // 2
    return min(max(i - hw, 0), npts - width)


def diff_matrix(npts: int, spacing: float, deriv: int, width: int, periodic: bool) -> sp.csr_matrix:
    """npts x npts matrix of the deriv-th derivative on a uniform line of spacing ``spacing``.

    Periodic lines use the centred window with wrap-around; other lines use the centred
    window where it fits and the shifted window of the same width near the ends.
    """
    if not periodic and npts < width:
        raise ValueError("line shorter than the stencil")
    rows, cols, vals = [], [], []
    hw = width // 2
    for i in range(npts):
        if periodic:
            offs = np.arange(-hw, hw + 1)
            w = fornberg(0.0, offs * spacing, deriv)[:, deriv]
            idx = (i + offs) % npts
        else:
            s = window_start(i, npts, width)
            idx = np.arange(s, s + width)
            w = fornberg(i * spacing, idx * spacing, deriv)[:, deriv]
        rows.extend([i] * width)
        cols.extend(idx.tolist())
        vals.extend(w.tolist())
    return sp.csr_matrix((vals, (rows, cols)), shape=(npts, npts))
