"""Fixed preconditioners built on the still-water operator (test infrastructure, see package header).

Sec. 3 left-preconditions GMRES with a fixed factorisation of the operator of an almost
still-water state (eta = 0), computed once per simulation. The role kept here: a fixed
linear map M^-1 built from the second-order still-water operator M of
``discretization.low_order_operator``. Two such maps (readings, not the paper's ILU):

* line Jacobi: z0 = 0, z_{s+1} = z_s + omega L^-1 (v - M z_s), nu sweeps, where L keeps the
  entries of M that couple nodes of the same vertical column (one column solve per sweep);
* V-cycle: one V(nu1, nu2) cycle with semicoarsening in x (coarse grid = every other
  column, nz unchanged, M rediscretised on the coarse grid), line-Jacobi smoothing,
  linear interpolation in x, full weighting in x for the residual (half/half at a wall
  column, injection at ghost columns), an exact solve on the coarsest grid. Coarsening
  stops at the first grid with at most ``coarse_max`` unknowns (or when the column count
  cannot be halved further).

Pins (tests/test_oracle_precond.py): line Jacobi with nu = 1, omega = 1 equals the exact
block-diagonal column solve (dense, brute force); a one-level V-cycle equals the exact
solve of M; the two-grid operators satisfy interpolation/restriction identities on
columns-constant fields; the V-cycle is a fixed linear map (linearity check).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretization import Grid, low_order_operator


def same_column_part(grid: Grid, m: sp.spmatrix) -> sp.csr_matrix:
    """Entries of m that couple two nodes of the same column."""
    coo = m.tocoo()
    keep = (coo.row % grid.ncol) == (coo.col % grid.ncol)
    return sp.csr_matrix((coo.data[keep], (coo.row[keep], coo.col[keep])), shape=m.shape)


class LineJacobi:
    def __init__(self, grid: Grid, m: sp.spmatrix, nu: int = 1, omega: float = 1.0):
        self.grid, self.m, self.nu, self.omega = grid, m.tocsr(), nu, omega
        self.lu = spla.splu(same_column_part(grid, m).tocsc())

    def sweep(self, z, v):
        return z + self.omega * self.lu.solve(v - self.m @ z)

    def __call__(self, v):
        z = np.zeros_like(v)
        for _ in range(self.nu):
            z = self.sweep(z, v)
        return z


def coarsen(grid: Grid, h_phys):
    """Next coarser grid (every other column) and its depth samples, or None."""
    if grid.periodic:
        if grid.ncol % 2 or grid.ncol // 2 < 4:
            return None
        return Grid(grid.ncol // 2 + 1, grid.nz, "periodic", grid.length), np.asarray(h_phys)[::2]
    if (grid.nx - 1) % 2 or (grid.nx - 1) // 2 + 1 < 3:
        return None
    return Grid((grid.nx - 1) // 2 + 1, grid.nz, "walls", grid.length), np.asarray(h_phys)[::2]


def interpolation(fine: Grid, coarse: Grid) -> sp.csr_matrix:
    """Linear interpolation in x of a coarse field onto the fine grid, level by level."""
    rows, cols, vals = [], [], []
    if fine.periodic:
        for c in range(fine.ncol):
            if c % 2 == 0:
                rows.append(c); cols.append(c // 2); vals.append(1.0)
            else:
                rows += [c, c]; cols += [(c - 1) // 2, ((c + 1) // 2) % coarse.ncol]; vals += [0.5, 0.5]
    else:
        for p in range(fine.nx):  # physical column p sits at index p + 1
            if p % 2 == 0:
                rows.append(p + 1); cols.append(p // 2 + 1); vals.append(1.0)
            else:
                rows += [p + 1, p + 1]; cols += [(p - 1) // 2 + 1, (p + 1) // 2 + 1]; vals += [0.5, 0.5]
        rows += [0, fine.ncol - 1]; cols += [0, coarse.ncol - 1]; vals += [1.0, 1.0]
    p1 = sp.csr_matrix((vals, (rows, cols)), shape=(fine.ncol, coarse.ncol))
    return sp.kron(sp.identity(fine.nl), p1, format="csr")


def restriction(fine: Grid, coarse: Grid) -> sp.csr_matrix:
    """Full weighting in x (1/4, 1/2, 1/4), rows summing to one, level by level."""
    rows, cols, vals = [], [], []
    if fine.periodic:
        for cc in range(coarse.ncol):
            c = 2 * cc
            rows += [cc] * 3; cols += [(c - 1) % fine.ncol, c, (c + 1) % fine.ncol]; vals += [0.25, 0.5, 0.25]
    else:
        for pc in range(coarse.nx):
            p = 2 * pc
            if pc == 0:
                rows += [1, 1]; cols += [1, 2]; vals += [0.5, 0.5]
            elif pc == coarse.nx - 1:
                rows += [pc + 1, pc + 1]; cols += [p + 1, p]; vals += [0.5, 0.5]
            else:
                rows += [pc + 1] * 3; cols += [p, p + 1, p + 2]; vals += [0.25, 0.5, 0.25]
        rows += [0, coarse.ncol - 1]; cols += [0, fine.ncol - 1]; vals += [1.0, 1.0]
    r1 = sp.csr_matrix((vals, (rows, cols)), shape=(coarse.ncol, fine.ncol))
    return sp.kron(sp.identity(fine.nl), r1, format="csr")


COARSE_MAX = 700


class VCycle:
    def __init__(self, grid: Grid, h_phys, nu1: int = 1, nu2: int = 1, omega: float = 1.0,
                 max_levels: int = 32, coarse_max: int = COARSE_MAX):
        self.nu1, self.nu2, self.omega = nu1, nu2, omega
        self.levels = []
        g, h = grid, np.asarray(h_phys, dtype=np.float64)
        while True:
            lev = dict(grid=g, m=low_order_operator(g, h))
            self.levels.append(lev)
            small = g.n <= coarse_max
            nxt = coarsen(g, h) if len(self.levels) < max_levels and not small else None
            if nxt is None:
                break
            gc, hc = nxt
            lev["P"] = interpolation(g, gc)
            lev["R"] = restriction(g, gc)
            g, h = gc, hc
        for lev in self.levels[:-1]:
            lev["smoother"] = LineJacobi(lev["grid"], lev["m"], 1, omega)
        self.coarse_lu = spla.splu(self.levels[-1]["m"].tocsc())

    def cycle(self, l: int, f):
        lev = self.levels[l]
        if l == len(self.levels) - 1:
            return self.coarse_lu.solve(f)
        sm = lev["smoother"]
        u = np.zeros_like(f)
        for _ in range(self.nu1):
            u = sm.sweep(u, f)
        r = f - lev["m"] @ u
        u = u + lev["P"] @ self.cycle(l + 1, lev["R"] @ r)
        for _ in range(self.nu2):
            u = sm.sweep(u, f)
        return u

    def __call__(self, v):
        return self.cycle(0, np.asarray(v, dtype=np.float64))


def make(grid: Grid, h_phys, kind: str = "mg", nu1: int = 1, nu2: int = 1, omega: float = 0.5,
         max_levels: int = 32, coarse_max: int = COARSE_MAX):
    """The fixed map M^-1 of a simulation: 'none', 'line' (nu1 sweeps), 'mg' or 'ilu0' (the
    paper's incomplete LU of the sixth-order operator at still water, oracle/ilu.py)."""
    if kind == "none":
        return lambda v: np.array(v, dtype=np.float64, copy=True)
    if kind == "line":
        return LineJacobi(grid, low_order_operator(grid, h_phys), nu1, omega)
    if kind == "mg":
        return VCycle(grid, h_phys, nu1, nu2, omega, max_levels, coarse_max)
    if kind == "ilu0":
        from .ilu import ILU0
        return ILU0(grid, h_phys)
    raise ValueError(kind)
