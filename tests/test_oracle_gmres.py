"""Pins of the oracle's GMRES against dense LU and textbook convergence facts."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import precond
from oracle.discretization import Grid, mixed_stage_operator
from oracle.gmres import NOCONV, OK, gmres
from paper_2511_18071_amd import workload as W


def _system(name="tiny_17x7", s=3):
    w = W.get(name)
    g = Grid(w.nx, w.nz, w.bc, w.length)
    ep, ec, ps = w.system(s)
    A = mixed_stage_operator(g, w.depth(), ep, ec)
    return w, g, A, A @ ps, ps


@pytest.mark.parametrize("pc", ["none", "line", "mg"])
def test_matches_dense_lu(pc):
    w, g, A, b, ps = _system()
    x_lu = np.linalg.solve(A.toarray(), b)
    minv = precond.make(g, w.depth(), pc)
    x, info = gmres(A, b, np.zeros(g.n), minv, 30, 1e-10)
    assert info.status == OK
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    cond = np.linalg.cond(A.toarray())
    assert np.linalg.norm(x - x_lu) <= 10 * cond * 1e-10 * np.linalg.norm(x_lu)
    assert np.linalg.norm(x_lu - ps) < 1e-12 * cond * np.linalg.norm(ps)


def test_diagonal_with_p_distinct_eigenvalues_converges_in_p_steps():
    n, p = 200, 7
    eig = np.repeat(np.arange(1.0, p + 1), n // p + 1)[:n]
    A = sp.diags(eig).tocsr()
    b = np.random.default_rng(0).standard_normal(n)
    x, info = gmres(A, b, np.zeros(n), lambda v: v.copy(), 30, 1e-12)
    assert info.status == OK and info.iters <= p and info.restarts == 0
    assert np.allclose(x, b / eig, rtol=1e-10)


def test_identity():
    n = 50
    A = sp.identity(n, format="csr")
    b = np.linspace(1, 2, n)
    x, info = gmres(A, b, np.zeros(n), lambda v: v.copy(), 10, 1e-12)
    assert info.iters == 1 and np.allclose(x, b)
    x, info = gmres(A, b, b.copy(), lambda v: v.copy(), 10, 1e-12)
    assert info.iters == 0 and info.relres0 == 0.0


def test_restarts_and_noconv():
    w, g, A, b, ps = _system()
    x_lu = np.linalg.solve(A.toarray(), b)
    minv = precond.make(g, w.depth(), "mg")
    x, info = gmres(A, b, np.zeros(g.n), minv, 4, 1e-8, max_restarts=500)
    assert info.status == OK and info.restarts >= 3
    assert 4 * info.restarts < info.iters <= 4 * (info.restarts + 1)
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
    assert np.linalg.norm(x - x_lu) <= 1e-4 * np.linalg.norm(x_lu)
    x, info = gmres(A, b, np.zeros(g.n), minv, 4, 1e-8, max_restarts=0)
    assert info.status == NOCONV and info.iters == 4 and info.restarts == 1
    assert info.relres < 1.0  # the best iterate of the cycle is returned


def test_zero_rhs():
    w, g, A, b, ps = _system()
    x, info = gmres(A, 0 * b, np.ones(g.n), lambda v: v.copy(), 10, 1e-8)
    assert np.all(x == 0) and info.iters == 0
