"""GPU parity of the sketch's forgetting in time (decay = SA_DECAY_TIME, Alg. 4's exponent
r^(tau_now - tau_l) in units of decay_dtau) against the oracle, through the C ABI.

Every system carries the time label of its stage (the LSERK45 stage times of the workload, a
non-uniform spacing); the sketch forgets by r to the time since the last stored solution. On
the small grids (seeds keep every oracle decision at least 3 % from its threshold) the
decisions are identical; on the bar the tie rule of the other sequence tests applies. The
sketch itself matches the oracle's to 1e-9; a checkpoint carries the time labels; the
argument errors are reported before any device work.
"""
import sys

import numpy as np
import pytest

from oracle.sequence import Simulation
from paper_2511_18071_amd import workload as W
from tests.parity_rules import check_decisions, margin_of, margins_text

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_2511_18071_amd import binding
    return binding


CASES = [("periodic_65x9", 15, 7), ("tiny_17x7", 12, 39), ("bar_513x17", 8, None)]


@pytest.mark.parametrize("name,nsys,seed", CASES)
def test_time_decay_sequence_parity(B, name, nsys, seed):
    w = W.get(name, seed=seed)
    kw = dict(decay="time", decay_dtau=w.dtau)
    _say(f"[decay time] {name} seed={seed} nsys={nsys} n={w.n}")
    ora = Simulation.from_workload(w, **kw)
    p = B.Problem.from_workload(w, stream=0, **kw)
    ties = 0
    for s in range(nsys):
        ep, ec, ps = w.system(s)
        tau = w.stage_times(s)[0]
        b = ora.operator(ep, ec) @ ps
        ro = ora.solve(ep, ec, b, tau=tau)
        p.set_surface(ep, ec)
        p.push_rhs(b)
        p.set_time(tau)
        info = p.solve()
        x = p.solution()
        dx = np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x)
        _say(f"   sys {s:2d} tau={tau:.4f}: gpu it={info.iters} ck={info.checks} rank={info.rank} | oracle "
             f"it={ro.info.iters} ck={ro.info.checks} rank={ro.rank} | dx={dx:.2e} | margin {margins_text(ro)}")
        assert info.status == 0 and info.relres <= w.rtol and dx <= 1e-7
        if check_decisions(info, ro, w.n, f"{name} decay time system {s}"):
            ties += 1
            _say(f"   tie at sys {s}: oracle margin {margin_of(ro):.2e}")
        assert ties <= 2
    p.close()


def test_time_decay_sketch_matches_oracle(B):
    w = W.get("periodic_65x9", seed=7)
    kw = dict(decay="time", decay_dtau=w.dtau)
    ora = Simulation.from_workload(w, **kw)
    p = B.Problem.from_workload(w, stream=0, **kw)
    for s in range(7):
        ep, ec, ps = w.system(s)
        b = ora.operator(ep, ec) @ ps
        ora.solve(ep, ec, b, tau=w.stage_times(s)[0])
        p.set_surface(ep, ec)
        p.push_rhs(b)
        p.set_time(w.stage_times(s)[0])
        p.solve()
    # reading the sketch stores the pending last solution first
    Y = p.sketch()
    assert p.sketch_count == 7 == ora.sketch.pushes
    assert np.abs(Y - ora.sketch.Y).max() <= 1e-9 * np.abs(ora.sketch.Y).max()
    p.close()


def test_time_decay_checkpoint_continues_bitwise(B):
    w = W.get("periodic_65x9", seed=7)
    kw = dict(decay="time", decay_dtau=w.dtau)
    systems = [w.system(s) for s in range(8)]
    taus = [w.stage_times(s)[0] for s in range(8)]
    ora = Simulation.from_workload(w)
    bs = [ora.operator(ep, ec) @ ps for ep, ec, ps in systems]

    def run(p, idx):
        out = []
        for s in idx:
            ep, ec, _ = systems[s]
            p.set_surface(ep, ec)
            p.push_rhs(bs[s])
            p.set_time(taus[s])
            info = p.solve()
            out.append((info.iters, info.checks, info.rank, p.solution()))
        return out

    full = B.Problem.from_workload(w, stream=0, **kw)
    ref = run(full, range(8))
    full.close()
    a = B.Problem.from_workload(w, stream=0, **kw)
    first = run(a, range(4))
    state = a.save_state()
    a.close()
    b = B.Problem.from_workload(w, stream=0, **kw)
    b.load_state(state)
    rest = run(b, range(4, 8))
    b.close()
    for (i1, c1, r1, x1), (i2, c2, r2, x2) in zip(ref, first + rest):
        assert (i1, c1, r1) == (i2, c2, r2)
        assert np.array_equal(x1, x2)


def test_time_decay_argument_errors(B):
    w = W.get("tiny_17x7")
    p = B.Problem.from_workload(w, stream=0, decay="time", decay_dtau=0.1)
    ep, ec, ps = w.system(0)
    p.set_surface(ep, ec)
    p.push_rhs(np.ones(w.n))
    with pytest.raises(B.SawaveError) as e:  # no time label
        p.solve()
    assert e.value.code == -1
    p.set_time(1.0)
    assert p.solve().status == 0
    with pytest.raises(B.SawaveError) as e:  # labels must not decrease
        p.set_time(0.5)
    assert e.value.code == -1
    p.close()
    q = B.Problem.from_workload(w, stream=0)
    with pytest.raises(B.SawaveError) as e:  # the problem counts solves
        q.set_time(1.0)
    assert e.value.code == -1
    q.close()
    for bad in (dict(decay="time", guess="range", window=8), dict(decay="time", decay_dtau=0.0)):
        with pytest.raises(B.SawaveError) as e:
            B.Problem.from_workload(w, stream=0, **bad)
        assert e.value.code == -1
    srv = B.Server(stream=0)
    with pytest.raises(B.SawaveError) as e:
        srv.open(w, decay="time")
    assert e.value.code == -1
    srv.close()
