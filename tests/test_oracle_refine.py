"""Pins of the oracle's mixed-precision refinement (dense LU, contraction, accuracy)."""
import numpy as np
import scipy.sparse as sp

from oracle import refine
from oracle.discretization import Grid, mixed_stage_operator
from oracle.precond import make
from paper_2511_18071_amd import workload as W


def _wellcond(n, seed):
    rs = np.random.default_rng(seed)
    A = np.eye(n) * 4.0 + rs.standard_normal((n, n)) / np.sqrt(n)
    return sp.csr_matrix(A), rs.standard_normal(n)


def test_exact_inner_cycle_is_one_direct_solve():
    A, b = _wellcond(60, 1)
    x, info = refine.solve(A, b, np.zeros(60), lambda v: np.array(v), m=60, rtol=1e-12, rtol_inner=1e-16,
                           inner=np.float64, use_trigger=False)
    ref = np.linalg.solve(A.toarray(), b)
    assert info.refinements == 1 and info.status == refine.OK
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_residual_contracts_by_the_inner_tolerance():
    A, b = _wellcond(200, 2)
    for tol in (1e-2, 1e-3):
        x, info = refine.solve(A, b, np.zeros(200), lambda v: np.array(v), m=40, rtol=1e-13, rtol_inner=tol,
                               use_trigger=False)
        h = [info.relres0] + info.history
        assert info.status == refine.OK and len(h) >= 3
        # kappa(A) u32 ~ 1e-7 << tol: every correction gains at least the inner tolerance (x10 slack)
        for a, c in zip(h[:-1], h[1:]):
            assert c <= 10.0 * tol * a, (tol, h)


def test_fp32_refinement_reaches_fp64_accuracy_on_the_mixed_stage_system():
    w = W.get("tiny_17x7")
    g = Grid(w.nx, w.nz, w.bc, w.length)
    ep, ec, ps = w.system(3)
    A = mixed_stage_operator(g, w.depth(), ep, ec)
    b = A @ ps
    minv = make(g, w.depth(), "mg")
    x, info = refine.solve(A, b, np.zeros(g.n), minv, m=10, rtol=1e-10)
    assert info.status == refine.OK and info.relres <= 1e-10
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    Ad = A.toarray()
    ref = np.linalg.solve(Ad, b)
    kappa = np.linalg.cond(Ad)
    assert np.linalg.norm(x - ref) <= 2.0 * kappa * 1e-10 * np.linalg.norm(ref)
    # the corrections are single precision: more than one is needed to get from 1 to 1e-10
    assert info.refinements >= 2


def test_fp64_inner_cycle_matches_gmres_decisions():
    # without rounding and with the floor out of reach the refinement path is GMRES(m)
    # with the same trigger rule: same iterations and residual checks
    from oracle import gmres
    w = W.get("tiny_17x7")
    g = Grid(w.nx, w.nz, w.bc, w.length)
    ep, ec, ps = w.system(2)
    A = mixed_stage_operator(g, w.depth(), ep, ec)
    b = A @ ps
    minv = make(g, w.depth(), "mg")
    x1, i1 = refine.solve(A, b, np.zeros(g.n), minv, m=10, rtol=1e-9, rtol_inner=1e-300, inner=np.float64)
    x2, i2 = gmres.gmres(A, b, np.zeros(g.n), minv, 10, 1e-9)
    assert (i1.iters, i1.checks) == (i2.iters, i2.checks)
    assert i1.refinements == i2.restarts + 1
    assert np.linalg.norm(x1 - x2) <= 1e-8 * np.linalg.norm(x2)
