"""Pins of the oracle's randomized range finder (Alg. 3) and its guess.

Against what the algorithm fixes, not against its own formula: the window forgets exactly
the solutions older than the K most recent ones; the sketch of a full-rank window has rank
min(k, K); V = Q and V = X Omega span the same space, so the least-squares guess is the same;
with k = K and a fixed operator the guess is Fischer's projection (Sec. 4: A x0 is the
orthogonal projection of b onto span(A X), computed here with numpy's least squares on the
unsketched window); a solution inside the window's span is found exactly (zero GMRES steps)."""
import numpy as np
import pytest

from oracle.discretization import Grid, mixed_stage_operator
from oracle.gmres import gmres
from oracle.rangefinder import RangeFinder
from oracle.sequence import Simulation
from oracle.subspace import guess
from paper_2511_18071_amd import workload as W


def _op(s=2):
    w = W.get("tiny_17x7")
    g = Grid(w.nx, w.nz, w.bc, w.length)
    ep, ec, ps = w.system(s)
    return w, g, mixed_stage_operator(g, w.depth(), ep, ec)


def test_window_forgets_exactly_the_oldest_solutions():
    n, K, k = 30, 6, 4
    rf = RangeFinder(n, K, k, seed=5)
    E = np.eye(n)
    for i in range(K + 3):  # unit vectors e_0 .. e_8: e_0, e_1, e_2 leave the window
        rf.push(E[i])
    V = rf.basis()
    assert np.all(V[:3] == 0.0)              # no trace of the forgotten solutions
    assert np.all(V[K + 3:] == 0.0)          # nothing outside the pushed ones
    assert np.linalg.matrix_rank(V[3:K + 3]) == k
    assert rf.X().shape == (n, K)


def test_sketch_rank_is_min_k_window():
    n = 50
    xs = np.random.default_rng(2).standard_normal((12, n))
    for K, k, pushed in ((10, 4, 12), (10, 10, 12), (10, 6, 3)):
        rf = RangeFinder(n, K, k, seed=1)
        for x in xs[:pushed]:
            rf.push(x)
        assert np.linalg.matrix_rank(rf.basis()) == min(k, K, pushed)


def test_q_and_sketch_give_the_same_guess():
    w, g, A = _op()
    xs = np.random.default_rng(3).standard_normal((8, g.n))
    b = np.random.default_rng(4).standard_normal(g.n)
    out = []
    for ortho in (False, True):
        rf = RangeFinder(g.n, 8, 5, seed=2, orthonormalize=ortho)
        for x in xs:
            rf.push(x)
        x0, rank = guess(A, rf.basis(), b)
        assert rank == 5
        out.append(x0)
    assert np.linalg.norm(out[0] - out[1]) <= 1e-10 * np.linalg.norm(out[1])


def test_q_is_orthonormal_and_spans_the_sketch():
    n = 60
    xs = np.random.default_rng(5).standard_normal((9, n))
    for K, k, pushed in ((8, 5, 9), (8, 6, 3)):
        a = RangeFinder(n, K, k, seed=4)
        q = RangeFinder(n, K, k, seed=4, orthonormalize=True)
        for x in xs[:pushed]:
            a.push(x)
            q.push(x)
        V, Q = a.basis(), q.basis()
        # a window of fewer solutions than k gives that many columns, not rounding noise
        assert Q.shape[1] == min(k, pushed)
        assert np.abs(Q.T @ Q - np.eye(Q.shape[1])).max() <= 1e-13
        assert np.linalg.norm(V - Q @ (Q.T @ V)) <= 1e-12 * np.linalg.norm(V)
        # ... and the same space as numpy's QR of the sketch when it has full rank
        if pushed >= k:
            Qn, _ = np.linalg.qr(V)
            assert np.linalg.norm(Qn - Q @ (Q.T @ Qn)) <= 1e-12 * np.linalg.norm(Qn)


def test_fischer_projection_when_k_equals_K():
    """Fixed A, k = K: span(X Omega) = span(X), so A x0 = argmin over span(A X) of ||. - b||."""
    w, g, A = _op()
    rs = np.random.default_rng(7)
    K = 6
    xs = rs.standard_normal((K, g.n))
    rf = RangeFinder(g.n, K, K, seed=9)
    for x in xs:
        rf.push(x)
    b = rs.standard_normal(g.n)
    x0, rank = guess(A, rf.basis(), b)
    B = A @ xs.T
    c, *_ = np.linalg.lstsq(B, b, rcond=None)
    assert rank == K
    assert np.linalg.norm(A @ x0 - B @ c) <= 1e-9 * np.linalg.norm(b)


def test_exact_guess_when_the_solution_is_in_the_window():
    w, g, A = _op()
    rs = np.random.default_rng(8)
    xs = rs.standard_normal((5, g.n))
    rf = RangeFinder(g.n, 5, 5, seed=3)
    for x in xs:
        rf.push(x)
    xt = xs.T @ rs.standard_normal(5)
    b = A @ xt
    x0, rank = guess(A, rf.basis(), b)
    assert np.linalg.norm(b - A @ x0) <= 1e-12 * np.linalg.norm(b)
    _, info = gmres(A, b, x0, lambda v: v, 10, 1e-10)
    assert info.iters == 0


def test_sequence_with_the_range_finder_converges_and_beats_cold():
    w = W.get("periodic_65x9")
    sims = {g: Simulation.from_workload(w, guess=g, window=12, k=6) for g in ("range", "cold")}
    its = {g: 0 for g in sims}
    for s in range(10):
        ep, ec, ps = w.system(s)
        b = sims["cold"].operator(ep, ec) @ ps
        for gm, sim in sims.items():
            r = sim.solve(ep, ec, b)
            assert r.info.status == 0 and r.info.relres <= w.rtol
            its[gm] += r.info.iters
    assert its["range"] < its["cold"]


def test_planted_mistake_is_caught():
    """A window that never forgets (the oldest solution kept) fails the forgetting pin."""
    class Leaky(RangeFinder):
        def push(self, x):
            super().push(x)
            self.K += 1  # the window grows: nothing is ever dropped

    rf = Leaky(30, 6, 4, seed=5)
    E = np.eye(30)
    for i in range(9):
        rf.push(E[i])
    assert not np.all(rf.basis()[:3] == 0.0)
