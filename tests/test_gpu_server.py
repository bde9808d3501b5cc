"""GPU tests of the continuous-batching server through the C ABI.

* every result is the same alone and in the mix: each simulation's sequence solved through
  the server, interleaved with other simulations of different sizes, precisions and guess
  modes, equals the same sequence solved alone through sa_solve with the same cluster size
  (identical decisions, every solution equal to 1e-13 relative: both run the same kernel
  code on the same inputs);
* device inputs produced on the server's stream by work still in flight at submit are read
  only after it (the request waits on an event recorded at submit);
* a simulation whose solve fails on the device (the abort flag of its bounded waits raised
  from the host) completes that request and every queued one with SA_EDEVICE, the others
  go on, the outstanding count drains and the simulation can be closed;
* admission queue: a simulation over the budget waits with its requests and runs once
  another one is closed;
* submit and poll from two host threads;
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
    xs = {}
    # interleave: system s of every simulation before system s + 1 of any
    for s in range(NSYS):
        for i, sid in enumerate(sims):
            ep, ec, b = systems[i][s]
            if mem == "device":
                ep, ec, b = (torch.from_numpy(v).cuda() for v in (ep, ec, b))
                x = torch.empty(works[i].n, dtype=torch.float64, device="cuda")
                keep.append((ep, ec, b))
            else:
                x = np.empty(works[i].n)
            xs[(i, s)] = x
            tickets[srv.submit(sid, ep, ec, b, x_out=x)] = (i, s)
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
        worst = 0.0
        for s in range(NSYS):
            x_mix = xs[(i, s)]
            x_mix = x_mix.cpu().numpy() if hasattr(x_mix, "cpu") else x_mix
            x_alone = alone[i][s][1]
            worst = max(worst, np.linalg.norm(x_mix - x_alone) / np.linalg.norm(x_alone))
        _say(f"   {name} {kw}: iters {[alone[i][s][0].iters for s in range(NSYS)]} | worst solution dx {worst:.1e}")
        assert worst <= 1e-13
    srv.close()


def test_server_fp64_results_match_the_oracle(B):
    w = W.get("periodic_65x9", seed=16)  # every oracle decision clear of its threshold by >= 3 %
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


def test_device_inputs_wait_for_the_producing_stream(B):
    """b is written on the server's stream behind a long chain of unrelated work and
    submitted without a synchronisation: the solve must see the final b."""
    import torch
    w = W.get("bar_65x9")
    systems = _systems(w, 3)
    alone = _alone(B, w, dict(cluster=2), systems)
    stream = torch.cuda.current_stream()
    srv = B.Server(stream=stream)
    sid = srv.open(w, cluster=2)
    keep, xs, tickets = [], [], []
    big = torch.randn(2048, 2048, dtype=torch.float64, device="cuda")
    for ep, ec, b in systems:
        e1, e2 = torch.from_numpy(ep).cuda(), torch.from_numpy(ec).cuda()
        bd = torch.zeros(w.n, dtype=torch.float64, device="cuda")
        bsrc = torch.from_numpy(b).cuda()
        torch.cuda.synchronize()
        acc = big
        for _ in range(20):  # tens of milliseconds of work ahead of the write of b
            acc = acc @ big * 1e-3
        bd.copy_(bsrc + 0.0 * acc[0, 0])
        x = torch.empty(w.n, dtype=torch.float64, device="cuda")
        tickets.append(srv.submit(sid, e1, e2, bd, x_out=x))
        keep.append((e1, e2, bd, bsrc))
        xs.append(x)
    got = {}
    while srv.outstanding > 0:
        for c in srv.poll(wait=True):
            got[c.ticket] = c
    for s, t in enumerate(tickets):
        assert got[t].info.status == 0
        assert got[t].info.iters == alone[s][0].iters
        x = xs[s].cpu().numpy()
        assert np.linalg.norm(x - alone[s][1]) <= 1e-13 * np.linalg.norm(alone[s][1])
    srv.close()


def test_device_failure_drains_the_simulation(B):
    w1, w2 = W.get("periodic_65x9"), W.get("bar_65x9")
    s1, s2 = _systems(w1, 3), _systems(w2, 2)
    srv = B.Server(stream=0)
    a = srv.open(w1, cluster=2)
    b = srv.open(w2, cluster=1)
    srv.debug_abort(a)  # its next solve ends at once with SA_EDEVICE
    ta = [srv.submit(a, *sy) for sy in s1]
    tb = [srv.submit(b, *sy) for sy in s2]
    got = {}
    polls = 0
    while srv.outstanding > 0:
        polls += 1
        assert polls < 100000
        for c in srv.poll(wait=True):
            got[c.ticket] = c
    _say(f"[server failure] statuses a {[got[t].info.status for t in ta]} b {[got[t].info.status for t in tb]}")
    assert all(got[t].info.status == -5 for t in ta)
    assert all(got[t].info.status == 0 for t in tb)
    with pytest.raises(B.SawaveError):
        srv.submit(a, *s1[0])
    srv.close_sim(a)
    srv.close_sim(b)
    assert srv.outstanding == 0 and srv.bytes_used == 0
    srv.close()


def test_admission_queue_runs_a_waiting_simulation_after_a_close(B):
    small = W.get("periodic_65x9")
    big = W.get("bar_513x17")
    fs, fb = B.footprint(small, cluster=1), B.footprint(big, cluster=1)
    srv = B.Server(stream=0, hbm_budget=fb + fs // 2, queue_admission=1)
    a = srv.open(big, cluster=1)
    b = srv.open(small, cluster=1)
    assert srv.admitted(a) == 1 and srv.admitted(b) == 0 and srv.bytes_used == fb
    sb = _systems(small, 2)
    tb = [srv.submit(b, *sy) for sy in sb]
    assert srv.poll(wait=True) == []  # nothing can run: b waits for memory
    assert srv.outstanding == 2
    srv.close_sim(a)
    assert srv.admitted(b) == 1 and srv.bytes_used == fs
    got = {}
    while srv.outstanding > 0:
        for c in srv.poll(wait=True):
            got[c.ticket] = c
    alone = _alone(B, small, dict(cluster=1), sb)
    assert [got[t].info.iters for t in tb] == [r[0].iters for r in alone]
    srv.close()


def test_submit_and_poll_from_two_threads(B):
    import threading
    import time
    works = [W.get("periodic_65x9"), W.get("bar_65x9")]
    systems = [_systems(w, 4) for w in works]
    alone = [_alone(B, w, dict(cluster=1), sy) for w, sy in zip(works, systems)]
    srv = B.Server(stream=0, max_inflight=2)
    sims = [srv.open(w, cluster=1) for w in works]
    tickets = {}
    lock = threading.Lock()

    def producer():
        for s in range(4):
            for i, sid in enumerate(sims):
                t = srv.submit(sid, *systems[i][s])
                with lock:
                    tickets[t] = (i, s)
                time.sleep(0.002)

    th = threading.Thread(target=producer)
    th.start()
    got = []
    deadline = time.time() + 120
    while len(got) < 8 and time.time() < deadline:
        got += srv.poll(wait=True, timeout_s=0.01)
    th.join()
    assert len(got) == 8
    order = {0: [], 1: []}
    for c in got:
        i, s = tickets[c.ticket]
        order[i].append(s)
        assert c.info.iters == alone[i][s][0].iters
    assert order[0] == [0, 1, 2, 3] and order[1] == [0, 1, 2, 3]
    srv.close()
