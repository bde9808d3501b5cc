"""GPU parity at the full size of the large single simulation: periodic 16385 x 33
(n = 557 056), GMRES(40), rank-16 EWMA guess, default cluster, through the C ABI.

* operator and preconditioner: every element against the FP64 oracle, with the bounds of the
  small cases (operator: 1e-11 of the row's |A||x|; preconditioner: max(1e-11, 8 kappa(M_c)
  eps) of max |z|, M_c the coarsest operator solved exactly);
* solves: the first two systems of the sequence (the first from an empty history) against
  the oracle's own sequence: identical decisions up to the tie rule of the small cases,
  relative residual <= rtol recomputed with the oracle's assembled operator, and solution
  difference <= 1e-7 relative.
"""
import sys

import numpy as np
import pytest

from oracle import precond as opc
from oracle.discretization import Grid, mixed_stage_operator
from oracle.sequence import Simulation
from paper_2511_18071_amd import workload as W
from tests.parity_rules import check_decisions, margins_text

pytestmark = pytest.mark.gpu

NAME = "periodic_16385x33"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_2511_18071_amd import binding
    return binding


def test_fullsize_operator_and_precond(B):
    w = W.get(NAME)
    _say(f"[fullsize operator+precond] {NAME} n={w.n}")
    g = Grid(w.nx, w.nz, w.bc, w.length)
    p = B.Problem.from_workload(w, stream=0)
    ep, ec, ps = w.system(1)
    A = mixed_stage_operator(g, w.depth(), ep, ec)
    p.set_surface(ep, ec)
    x = np.random.default_rng(17).standard_normal(w.n)
    y = p.apply_operator(x)
    bound = abs(A) @ np.abs(x)
    bound = np.maximum(bound, 1e-4 * bound.max())
    ratio = (np.abs(y - A @ x) / bound).max()
    _say(f"   operator: max err/(|A||x|) {ratio:.3e}")
    assert ratio <= 1e-11
    minv = opc.make(g, w.depth(), "mg", 1, w.nu2, coarse_max=w.coarse_max)  # the workload's V(1, nu2), as the problem
    kappa = np.linalg.cond(minv.levels[-1]["m"].toarray())
    tol = max(1e-11, 8.0 * kappa * np.finfo(float).eps)
    for v in (x, ps):
        z = p.apply_precond(v)
        ref = minv(v)
        err = np.abs(z - ref).max() / np.abs(ref).max()
        _say(f"   precond: rel err {err:.3e} (tol {tol:.1e})")
        assert err <= tol
    p.close()


def test_fullsize_solves(B):
    w = W.get(NAME)
    _say(f"[fullsize solves] {NAME} n={w.n}, 2 systems (oracle about a minute each)")
    ora = Simulation.from_workload(w)
    p = B.Problem.from_workload(w, stream=0)
    ties = 0
    for s in range(2):
        ep, ec, ps = w.system(s)
        A = ora.operator(ep, ec)
        b = A @ ps
        ro = ora.solve(ep, ec, b)
        p.set_surface(ep, ec)
        p.push_rhs(b)
        info = p.solve()
        x = p.solution()
        relres = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        dx = np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x)
        _say(f"   sys {s}: gpu it={info.iters} rs={info.restarts} ck={info.checks} rank={info.rank} "
             f"relres={info.relres:.3e} (oracle operator {relres:.3e}) | oracle it={ro.info.iters} "
             f"rs={ro.info.restarts} ck={ro.info.checks} rank={ro.rank} | dx={dx:.2e}")
        _say(f"   oracle margins {margins_text(ro)}")
        assert info.status == 0
        if check_decisions(info, ro, w.n, f"{NAME} system {s}"):
            ties += 1
        assert ties <= 1
        assert relres <= w.rtol * (1 + 1e-6)
        assert dx <= 1e-7
    p.close()
