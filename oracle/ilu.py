"""Incomplete LU factorisation with zero fill of the still-water operator (test infrastructure,
see package header).

Sec. 3 left-preconditions GMRES with a fixed incomplete LU factorisation of the operator of an
almost still-water state, built once per simulation by setting eta = 0 when the system is
generated (the flume runs of Sec. 5.2 use the same). This module is that preconditioner for
the sixth-order mixed-stage operator A(0, 0) of discretization.py (both stages at still water)
in the natural ordering of the unknowns (level-major, chi fastest).

ILU(0) (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Sec. 10.3): a unit lower
triangular L and an upper triangular U whose non-zero patterns are the strictly lower and the
upper part of A's pattern, such that (L U)_ij = a_ij wherever a_ij is in A's pattern.
Reading: A's pattern is structural, every node pair the composed seven-point stencils couple
(a coefficient that vanishes at still water, such as sigma_x on a flat bed or at the surface,
keeps its place), so that the factorisation does not depend on which sums cancel in rounding. Computed
row by row (the IKJ order): for row i and each k < i in the row's pattern, in increasing k,
l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj for every j > k of row k that is in row i's
pattern. The map applied is z = U^-1 (L^-1 v) by forward and backward substitution.

Pins (tests/test_oracle_ilu.py): on a matrix whose elimination creates no fill (banded
tridiagonal, or a matrix with a full pattern) ILU(0) is the exact LU (dense Doolittle); on the
still-water operator (L U)_ij = a_ij over A's pattern, L unit lower and U upper inside the
pattern; the apply solves (L U) z = v.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretization import Grid, _assemble, mixed_stage_operator
from .fd import diff_matrix


def structural_pattern(grid: Grid, width: int = 7) -> sp.csr_matrix:
    """Every (row, column) the composed operator's stencils reach, as a 0/1 CSR matrix: the
    mixed-stage form of discretization.mixed_stage_operator with every weight and coefficient
    replaced by one (no sum can cancel)."""
    def ones(m):
        m = sp.csr_matrix(m, copy=True)
        m.data[:] = 1.0
        return m
    dx = grid.along_x(ones(diff_matrix(grid.ncol, grid.dx, 1, width, grid.periodic)))
    ds = grid.along_sigma(ones(diff_matrix(grid.nl, grid.dsig, 1, width, False)))
    gchi = dx + ds
    pde = dx @ gchi + ds @ gchi + ds @ ds
    a = abs(_assemble(grid, pde, gchi, ds, np.ones(grid.ncol)))
    a.data[:] = 1.0
    a.sort_indices()
    return a


def ilu0(a: sp.spmatrix, pattern: sp.spmatrix | None = None):
    """(L, U) of ILU(0): L unit lower (diagonal stored), U upper, both CSR on the pattern
    (A's stored entries when none is given; a given pattern must contain them)."""
    a = sp.csr_matrix(a, dtype=np.float64, copy=True)
    a.sum_duplicates()
    a.sort_indices()
    n = a.shape[0]
    if pattern is not None:
        p = sp.csr_matrix(pattern, copy=True)
        p.sort_indices()
        ptr, ind = p.indptr.astype(np.int64), p.indices.astype(np.int64)
        val = np.zeros(ind.size)
        where = np.full(n, -1, dtype=np.int64)
        for i in range(n):
            where[ind[ptr[i]:ptr[i + 1]]] = np.arange(ptr[i], ptr[i + 1])
            cols = a.indices[a.indptr[i]:a.indptr[i + 1]]
            pos = where[cols]
            if np.any(pos < 0):
                raise ValueError(f"row {i} of A reaches outside the pattern")
            val[pos] = a.data[a.indptr[i]:a.indptr[i + 1]]
            where[ind[ptr[i]:ptr[i + 1]]] = -1
    else:
        ptr, ind, val = a.indptr, a.indices, a.data
    diag = np.empty(n, dtype=np.int64)
    for i in range(n):
        row = ind[ptr[i]:ptr[i + 1]]
        p = np.searchsorted(row, i)
        if p >= row.size or row[p] != i:
            raise ValueError(f"row {i} has no diagonal entry")
        diag[i] = ptr[i] + p
    where = np.full(n, -1, dtype=np.int64)  # position of column j in the current row, or -1
    for i in range(n):
        lo, hi = ptr[i], ptr[i + 1]
        where[ind[lo:hi]] = np.arange(lo, hi)
        for kk in range(lo, diag[i]):
            k = ind[kk]
            piv = val[diag[k]]
            if piv == 0.0:
                raise ZeroDivisionError(f"zero pivot at row {k}")
            val[kk] /= piv
            lik = val[kk]
            ks, ke = diag[k] + 1, ptr[k + 1]
            cols = ind[ks:ke]
            pos = where[cols]
            hit = pos >= 0
            val[pos[hit]] -= lik * val[ks:ke][hit]
        where[ind[lo:hi]] = -1
    rows = np.repeat(np.arange(n), np.diff(ptr))
    lower = ind < rows
    L = sp.csr_matrix((val[lower], (rows[lower], ind[lower])), shape=(n, n)) + sp.identity(n, format="csr")
    upper = ~lower
    U = sp.csr_matrix((val[upper], (rows[upper], ind[upper])), shape=(n, n))
    return L.tocsr(), U.tocsr()


class ILU0:
    """The fixed map z = (L U)^-1 v of the still-water operator A(0, 0)."""

    def __init__(self, grid: Grid, h_phys):
        zero = np.zeros(grid.nx - 1 if grid.periodic else grid.nx)
        self.a = mixed_stage_operator(grid, h_phys, zero, zero)
        self.pattern = structural_pattern(grid)
        self.L, self.U = ilu0(self.a, self.pattern)

    def __call__(self, v):
        y = spla.spsolve_triangular(self.L, np.asarray(v, dtype=np.float64), lower=True, unit_diagonal=True)
        return spla.spsolve_triangular(self.U, y, lower=False)
