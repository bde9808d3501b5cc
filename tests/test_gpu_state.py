"""Checkpoint and restore of the solver state (sa_save_state / sa_load_state) through the C
ABI: a problem restored mid-sequence continues exactly like the uninterrupted one (Alg. 4's
sketch, or Alg. 3's window and rows of Omega, plus the last solution and the counters that
position the sketch's random stream): the same decisions and bitwise the same solutions and
sketch, for the EWMA and the range-finder guesses; a state is refused by a problem of other
sketch options."""
import sys

import numpy as np
import pytest

from oracle.sequence import Simulation
from paper_2511_18071_amd import workload as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_2511_18071_amd import binding
    return binding


@pytest.mark.parametrize("name,kw", [("bar_65x9", dict()), ("periodic_257x33", dict()),
                                     ("bar_65x9", dict(guess="range", window=8, k=5)),
                                     ("bar_65x9", dict(precision="fp32_ir", rtol=1e-10))])
def test_restored_problem_continues_exactly(B, name, kw):
    w = W.get(name)
    ora = Simulation.from_workload(w)
    systems = []
    for s in range(10):
        ep, ec, ps = w.system(s)
        systems.append((ep, ec, ora.operator(ep, ec) @ ps))
    a = B.Problem.from_workload(w, stream=0, **kw)
    for ep, ec, b in systems[:6]:
        a.set_surface(ep, ec)
        a.push_rhs(b)
        a.solve()
    state = a.save_state()
    _say(f"[state] {name} {kw}: {len(state)} bytes after 6 solves")
    r = B.Problem.from_workload(w, stream=0, **kw)
    r.load_state(state)
    for s, (ep, ec, b) in enumerate(systems[6:], start=6):
        out = []
        for p in (a, r):
            p.set_surface(ep, ec)
            p.push_rhs(b)
            info = p.solve()
            out.append((info, p.solution()))
        (ia, xa), (ir, xr) = out
        _say(f"   sys {s}: uninterrupted it={ia.iters} rank={ia.rank} | restored it={ir.iters} rank={ir.rank}")
        assert (ia.iters, ia.restarts, ia.refinements, ia.checks, ia.rank, ia.status) == \
            (ir.iters, ir.restarts, ir.refinements, ir.checks, ir.rank, ir.status)
        assert ia.relres0 == ir.relres0 and ia.relres == ir.relres
        assert np.array_equal(xa, xr)
    if kw.get("guess", "ewma") == "ewma":
        assert np.array_equal(a.sketch(), r.sketch())
        assert a.sketch_count == r.sketch_count
    a.close()
    r.close()


def test_state_of_other_options_is_refused(B):
    w = W.get("bar_65x9")
    a = B.Problem.from_workload(w, stream=0)
    ep, ec, ps = w.system(0)
    b = Simulation.from_workload(w).operator(ep, ec) @ ps
    a.set_surface(ep, ec)
    a.push_rhs(b)
    a.solve()
    state = a.save_state()
    for bad in (dict(k=w.k - 1), dict(guess="range", window=8), dict(seed=w.seed + 1)):
        other = B.Problem.from_workload(w, stream=0, **bad)
        with pytest.raises(B.SawaveError) as e:
            other.load_state(state)
        assert e.value.code == -1
        other.close()
    with pytest.raises(B.SawaveError):
        a.load_state(state[:-8])
    a.close()
