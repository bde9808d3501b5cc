"""GPU tests of the continuous-batching server through the C ABI.

* every result is the same alone and in the mix: each simulation's sequence solved through
  the server, interleaved with other simulations of different sizes, precisions and guess
  modes, equals the same sequence solved alone through sa_solve with the same cluster size
  (identical decisions, solutions equal to 1e-13 relative: both run the same kernel code on
  the same inputs);
* the FP64 results also match the oracle (decisions and 1e-7 solution bar, as in the
  single-problem parity tests);
* requests of one simulation complete in submission order; host and device inputs;
* admission by HBM footprint: a simulation that does not fit the budget is refused (nothing
  allocated) and admitted once another one is closed.
"""
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


MIX = [
    ("tiny_17x7", dict(cluster=1)),
    ("periodic_65x9", dict(cluster=2)),
    ("bar_65x9", dict(cluster=1, precision="fp32_ir", rtol=1e-10)),
    ("bar_513x17", dict(cluster=4)),
    ("periodic_65x9", dict(cluster=1, guess="cold")),
    ("bar_65x9", dict(cluster=3, guess="previous")),
]
NSYS = 6


def _systems(w, n):
    out = []
    ora = Simulation.from_workload(w)
    for s in range(n):
        ep, ec, ps = w.system(s)
        out.append((ep, ec, ora.operator(ep, ec) @ ps))
    return out


def _alone(B, w, kw, systems):
    p = B.Problem.from_workload(w, stream=0, **kw)
    res = []
    for ep, ec, b in systems:
        p.set_surface(ep, ec)
        p.push_rhs(b)
        info = p.solve()
        res.append((info, p.solution()))
    p.close()
    return res


@pytest.mark.parametrize("mem", ["host", "device"])
def test_results_alone_equal_results_in_the_mix(B, mem):
    import torch
    _say(f"[server mix] {len(MIX)} simulations x {NSYS} systems, {mem} inputs")
    works = [W.get(name) for name, _ in MIX]
    systems = [_systems(w, NSYS) for w in works]
    alone = [_alone(B, w, kw, sy) for w, (_, kw), sy in zip(works, MIX, systems)]
    srv = B.Server(stream=0, max_inflight=2)
    sims = [srv.open(w, **kw) for w, (_, kw) in zip(works, MIX)]
    assert all(s is not None for s in sims)
    keep = []
    tickets = {}
    # interleave: system s of every simulation before system s + 1 of any
    for s in range(NSYS):
        for i, sid in enumerate(sims):
            ep, ec, b = systems[i][s]
            if mem == "device":
                ep, ec, b = (torch.from_numpy(v).cuda() for v in (ep, ec, b))
                keep.append((ep, ec, b))
            tickets[srv.submit(sid, ep, ec, b)] = (i, s)
    done = {}
    order = {i: [] for i in range(len(sims))}
    while srv.outstanding > 0:
        for c in srv.poll(wait=True):
            i, s = tickets[c.ticket]
            done[(i, s)] = c
            order[i].append(s)
    for i in range(len(sims)):
        assert order[i] == list(range(NSYS)), order[i]  # FIFO per simulation
    for i, (name, kw) in enumerate(MIX):
        for s in range(NSYS):
            a, c = alone[i][s][0], done[(i, s)].info
            assert c.status == 0, (name, s, c)
            assert (c.iters, c.restarts, c.refinements, c.checks, c.rank) == \
                (a.iters, a.restarts, a.refinements, a.checks, a.rank), (name, kw, s, c, a)
        x_mix = srv.solution(sims[i])
        x_alone = alone[i][-1][1]
        dx = np.linalg.norm(x_mix - x_alone) / np.linalg.norm(x_alone)
        _say(f"   {name} {kw}: iters {[alone[i][s][0].iters for s in range(NSYS)]} | last solution dx {dx:.1e}")
        assert dx <= 1e-13
    srv.close()


def test_server_fp64_results_match_the_oracle(B):
    w = W.get("periodic_65x9")
    systems = _systems(w, 8)
    ora = Simulation.from_workload(w)
    srv = B.Server(stream=0)
    sid = srv.open(w, cluster=2)
    t = [srv.submit(sid, ep, ec, b) for ep, ec, b in systems]
    got = {}
    while srv.outstanding > 0:
        for c in srv.poll(wait=True):
            got[c.ticket] = c
    for s, (ep, ec, b) in enumerate(systems):
        ro = ora.solve(ep, ec, b)
        c = got[t[s]].info
        assert (c.iters, c.restarts, c.checks, c.rank) == (ro.info.iters, ro.info.restarts, ro.info.checks, ro.rank)
    x = srv.solution(sid)
    assert np.linalg.norm(x - ro.x) <= 1e-7 * np.linalg.norm(ro.x)
    srv.close()


def test_admission_by_hbm_footprint(B):
    small = W.get("periodic_65x9")
    big = W.get("bar_513x17")
    fs, fb = B.footprint(small, cluster=1), B.footprint(big, cluster=1)
    _say(f"[server admission] footprints {fs} and {fb} bytes")
    srv = B.Server(stream=0, hbm_budget=fb + fs // 2)
    a = srv.open(big, cluster=1)
    assert a is not None and srv.bytes_used == fb
    assert srv.open(small, cluster=1) is None  # refused, nothing allocated
    assert srv.bytes_used == fb
    srv.close_sim(a)
    assert srv.bytes_used == 0
    b = srv.open(small, cluster=1)
    assert b is not None and srv.bytes_used == fs
    ep, ec, ps = small.system(0)
    bb = Simulation.from_workload(small).operator(ep, ec) @ ps
    srv.submit(b, ep, ec, bb)
    with pytest.raises(B.SawaveError):
        srv.close_sim(b)  # still has work
    while srv.outstanding > 0:
        srv.poll(wait=True)
    srv.close_sim(b)
    srv.close()
