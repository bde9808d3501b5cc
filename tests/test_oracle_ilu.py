"""Pins of the oracle's ILU(0) (oracle/ilu.py) against what the definition fixes.

* Where elimination creates no fill (a tridiagonal matrix; a matrix whose pattern is full)
  ILU(0) is the exact LU factorisation without pivoting, computed here by the textbook dense
  Doolittle recurrence.
* On the sixth-order still-water operator of the solver (the factorisation the solver uses),
  (L U)_ij = a_ij at every (i, j) of A's structural pattern (Saad, Sec. 10.3), L is unit lower
  triangular and U upper triangular inside the pattern, and the entries of L U outside the
  pattern (the dropped fill) are not all zero, so the factorisation really is incomplete.
* The map solves (L U) z = v.
A skipped update, a wrong elimination order or a pivot taken from the wrong row breaks the
pattern identity or the exact-LU cases.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.discretization import Grid, mixed_stage_operator
from oracle.ilu import ILU0, ilu0
from paper_2511_18071_amd import workload as W


def _doolittle(a):
    n = a.shape[0]
    L, U = np.eye(n), np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            U[i, j] = a[i, j] - L[i, :i] @ U[:i, j]
        for j in range(i + 1, n):
            L[j, i] = (a[j, i] - L[j, :i] @ U[:i, i]) / U[i, i]
    return L, U


def test_tridiagonal_is_exact_lu():
    rng = np.random.default_rng(1)
    n = 40
    a = sp.diags([rng.uniform(-1, 1, n - 1), 4 + rng.uniform(0, 1, n), rng.uniform(-1, 1, n - 1)], [-1, 0, 1])
    L, U = ilu0(a)
    Ld, Ud = _doolittle(a.toarray())
    assert np.allclose(L.toarray(), Ld, rtol=0, atol=1e-14)
    assert np.allclose(U.toarray(), Ud, rtol=0, atol=1e-13)


def test_full_pattern_is_exact_lu():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((12, 12)) + 12 * np.eye(12)
    L, U = ilu0(sp.csr_matrix(a))
    Ld, Ud = _doolittle(a)
    assert np.allclose(L.toarray(), Ld, atol=1e-13) and np.allclose(U.toarray(), Ud, atol=1e-12)


@pytest.mark.parametrize("name", ["tiny_17x7", "bar_65x9", "periodic_65x9"])
def test_still_water_factorisation_matches_a_on_its_pattern(name):
    w = W.get(name)
    g = Grid(w.nx, w.nz, w.bc, w.length)
    m = ILU0(g, w.depth())
    zero = np.zeros(w.nphys)
    a = mixed_stage_operator(g, w.depth(), zero, zero).tocsr()
    assert abs(m.a - a).max() == 0.0
    L, U = m.L, m.U
    assert abs(sp.tril(L, -1) - (L - sp.identity(g.n))).max() == 0.0 and np.all(L.diagonal() == 1.0)
    assert abs(sp.triu(U) - U).max() == 0.0
    pat = m.pattern
    assert (abs(a) - abs(a).multiply(pat)).nnz == 0  # the structural pattern holds A's entries
    # L and U stay inside A's pattern
    assert (sp.csr_matrix(abs(L - sp.identity(g.n))) - sp.csr_matrix(abs(L - sp.identity(g.n))).multiply(pat)).nnz == 0
    assert (sp.csr_matrix(abs(U)) - sp.csr_matrix(abs(U)).multiply(pat)).nnz == 0
    lu = (L @ U).tocsr()
    on = lu.multiply(pat) - a
    scale = abs(a).max()
    assert abs(on).max() <= 1e-12 * scale
    off = (lu - lu.multiply(pat))
    assert abs(off).max() > 1e-6 * scale  # fill was dropped: an incomplete factorisation


def test_apply_solves_lu_system():
    w = W.get("bar_65x9")
    g = Grid(w.nx, w.nz, w.bc, w.length)
    m = ILU0(g, w.depth())
    v = np.random.default_rng(3).standard_normal(g.n)
    z = m(v)
    r = m.L @ (m.U @ z) - v
    # backward stability of the two substitutions: r_i within a few eps of (|L| |U| |z|)_i
    bound = abs(m.L) @ (abs(m.U) @ np.abs(z))
    assert np.all(np.abs(r) <= 1e-13 * bound + 1e-15)
