"""GPU edge cases through the C ABI, each against the FP64 oracle's own outcome:

* a zero right-hand side: x = 0 exactly, no iterations, status OK (the oracle's GMRES returns
  the zero vector before any step), in FP64 and with FP32 refinement (whose inner iteration
  counts are not compared on the ordinary systems before it: the two sides round differently);
* a system solved twice in a row: the second time the solution lies in the span of the
  sketch (the exact-guess case of the subspace guess), so both sides accept the guess on the
  initial residual (row a8) with the same decisions;
* the restart cap: GMRES(4) with no restart allowed on a system that needs more stops with
  SA_NOCONV after exactly four steps on both sides, with the same residual to 1e-9 relative;
* a one-column-wide ragged last tile on every level of a cluster solve (walls, 133 columns).
"""
import sys

import numpy as np
import pytest

from oracle.sequence import Simulation
from paper_2511_18071_amd import workload as W
from tests.parity_rules import check_decisions, margins_text

pytestmark = pytest.mark.gpu

SA_NOCONV = 1


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_2511_18071_amd import binding
    return binding


@pytest.mark.parametrize("name,kw", [("bar_65x9", {}), ("periodic_65x9", dict(precision="fp32_ir", rtol=1e-10))])
def test_zero_rhs(B, name, kw):
    w = W.get(name, seed=41 if name == "bar_65x9" else None)  # clear decisions (>= 3 % margins)
    _say(f"[edge zero rhs] {name} {kw}")
    ora = Simulation.from_workload(w, **kw)
    p = B.Problem.from_workload(w, stream=0, cluster=2, **kw)
    for s in range(3):  # after two ordinary solves, so the sketch is not empty
        ep, ec, ps = w.system(s)
        b = ora.operator(ep, ec) @ ps if s < 2 else np.zeros(w.n)
        ro = ora.solve(ep, ec, b)
        p.set_surface(ep, ec)
        p.push_rhs(b)
        info = p.solve()
        x = p.solution()
        _say(f"   sys {s}: gpu it={info.iters} status={info.status} | oracle it={ro.info.iters}")
        assert info.status == 0
        if kw.get("precision") != "fp32_ir":  # the FP32 inner steps round differently on the two sides
            assert info.iters == ro.info.iters
        if s == 2:
            assert info.iters == 0 and np.all(x == 0.0) and np.all(ro.x == 0.0)
    p.close()


def test_repeated_system_accepts_the_guess(B):
    w = W.get("bar_65x9", seed=41)  # clear decisions (>= 3 % margins)
    _say("[edge repeated system] bar_65x9")
    ora = Simulation.from_workload(w)
    p = B.Problem.from_workload(w, stream=0, cluster=3)
    seq = [0, 1, 2, 2]
    for s in seq:
        ep, ec, ps = w.system(s)
        b = ora.operator(ep, ec) @ ps
        ro = ora.solve(ep, ec, b)
        p.set_surface(ep, ec)
        p.push_rhs(b)
        info = p.solve()
        _say(f"   sys {s}: gpu it={info.iters} rank={info.rank} r0={info.relres0:.2e} | oracle it={ro.info.iters} "
             f"rank={ro.rank} r0={ro.info.relres0:.2e}")
        assert (info.iters, info.restarts, info.checks, info.rank) == \
            (ro.info.iters, ro.info.restarts, ro.info.checks, ro.rank)
    assert info.iters == 0 and info.relres0 <= w.rtol


def test_restart_cap_gives_noconv(B):
    w = W.get("bar_65x9")
    kw = dict(restart=4, max_restarts=0, guess="cold")
    _say(f"[edge restart cap] bar_65x9 {kw}")
    ora = Simulation.from_workload(w, **kw)
    p = B.Problem.from_workload(w, stream=0, cluster=2, **kw)
    ep, ec, ps = w.system(0)
    b = ora.operator(ep, ec) @ ps
    ro = ora.solve(ep, ec, b)
    p.set_surface(ep, ec)
    p.push_rhs(b)
    info = p.solve()
    _say(f"   gpu status={info.status} it={info.iters} rs={info.restarts} relres={info.relres:.6e} | oracle "
         f"status={ro.info.status} it={ro.info.iters} rs={ro.info.restarts} relres={ro.info.relres:.6e}")
    assert info.status == SA_NOCONV and ro.info.status == SA_NOCONV
    assert (info.iters, info.restarts) == (ro.info.iters, ro.info.restarts) == (4, 1)
    assert abs(info.relres - ro.info.relres) <= 1e-9 * ro.info.relres
    p.close()


def test_ragged_single_column_tiles(B):
    w = W.get("bar_65x9")
    w.nx = 131  # 133 columns with the ghosts: 4 tiles of 32 and one of 5 on level 0
    _say(f"[edge ragged tiles] walls nx={w.nx}")
    ora = Simulation.from_workload(w)
    p = B.Problem.from_workload(w, stream=0)  # default cluster: one 32-column tile each
    for s in range(4):
        ep, ec, ps = w.system(s)
        b = ora.operator(ep, ec) @ ps
        ro = ora.solve(ep, ec, b)
        p.set_surface(ep, ec)
        p.push_rhs(b)
        info = p.solve()
        x = p.solution()
        dx = np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x)
        _say(f"   sys {s}: gpu it={info.iters} ck={info.checks} rank={info.rank} | oracle it={ro.info.iters} "
             f"ck={ro.info.checks} rank={ro.rank} | dx={dx:.2e} | margin {margins_text(ro)}")
        assert info.status == 0 and info.relres <= w.rtol and dx <= 1e-7
        check_decisions(info, ro, w.n, f"ragged walls nx={w.nx} system {s}")
    p.close()
