"""Pins of the oracle's EWMA sketch, least-squares guess and random stream."""
import numpy as np
import pytest

from oracle import rng
from oracle.discretization import Grid, mixed_stage_operator
from oracle.gmres import gmres
from oracle.sequence import Simulation
from oracle.subspace import EWMASketch, guess, householder_lstsq_drop
from paper_2511_18071_amd import workload as W


def test_splitmix64_published_first_output():
    # SplitMix64 seeded with 0: first output 0xE220A8397B1DCDAF (Steele, Lea & Flood 2014)
    assert rng.splitmix64(0, 1) == 0xE220A8397B1DCDAF


def test_gaussian_stream_moments():
    z = np.array([rng.gaussian(11, s, a) for s in range(1024) for a in range(64)])
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.03
    assert rng.omega(11, 5, 3) == [rng.gaussian(11, 5, a) for a in range(3)]


def test_streaming_equals_weighted_sum():
    n, k, r, seed = 40, 5, 0.8, 3
    xs = np.random.default_rng(0).standard_normal((9, n))
    sk = EWMASketch(n, k, r, seed)
    for x in xs:
        sk.push(x)
    ref = sum(r ** (len(xs) - 1 - l) * np.outer(xs[l], rng.omega(seed, l, k)) for l in range(len(xs)))
    assert np.allclose(sk.Y, ref, rtol=1e-13, atol=1e-13)


def test_time_decay_equals_weighted_sum_over_time_labels():
    """Alg. 4 with the exponent in time: Y = sum_l r^((tau_last - tau_l) / dtau) x_l omega_l^T
    for non-uniform labels (the LSERK45 stage times of three steps); a recursion that took the
    time since the first solution, or the label itself, instead of the time since the last
    stored one fails this."""
    n, k, r, seed, dt = 30, 4, 0.7, 5, 0.025
    w = W.get("bar_65x9")
    taus = [w.stage_times(s)[0] for s in range(15)]
    assert len(set(np.round(np.diff(taus), 12))) > 2  # the stage spacing is not uniform
    xs = np.random.default_rng(1).standard_normal((len(taus), n))
    sk = EWMASketch(n, k, r, seed, decay_dtau=dt)
    for x, t in zip(xs, taus):
        sk.push(x, t)
    ref = sum(r ** ((taus[-1] - taus[l]) / dt) * np.outer(xs[l], rng.omega(seed, l, k)) for l in range(len(xs)))
    assert np.allclose(sk.Y, ref, rtol=1e-12, atol=1e-13)


def test_time_decay_with_unit_spacing_is_the_per_solve_decay():
    n, k, r, seed = 25, 3, 0.85, 2
    xs = np.random.default_rng(2).standard_normal((7, n))
    a, b = EWMASketch(n, k, r, seed), EWMASketch(n, k, r, seed, decay_dtau=2.0)
    for i, x in enumerate(xs):
        a.push(x)
        b.push(x, 2.0 * i + 10.0)
    assert np.array_equal(a.Y, b.Y)


def _op(s=2):
    w = W.get("tiny_17x7")
    g = Grid(w.nx, w.nz, w.bc, w.length)
    ep, ec, ps = w.system(s)
    return w, g, mixed_stage_operator(g, w.depth(), ep, ec)


def test_guess_equals_dense_least_squares_projection():
    w, g, A = _op()
    rs = np.random.default_rng(1)
    Y = rs.standard_normal((g.n, 6))
    b = rs.standard_normal(g.n)
    x0, rank = guess(A, Y, b)
    W_ = A @ Y
    z, *_ = np.linalg.lstsq(W_, b, rcond=None)
    ref = Y @ z
    assert rank == 6
    assert np.linalg.norm(A @ x0 - A @ ref) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x0 - ref) <= 1e-8 * np.linalg.norm(ref)


def test_exact_guess_when_solution_in_span_of_history():
    """Thm. 4.1 with epsilon = 0: x(t) in span(X) gives a guess with zero residual (Sec. 4.2)."""
    w, g, A = _op(5)
    rs = np.random.default_rng(2)
    sk = EWMASketch(g.n, 6, 0.9, 7)
    hist = rs.standard_normal((6, g.n))
    for x in hist:
        sk.push(x)
    c = rs.standard_normal(6)
    xt = c @ hist
    b = A @ xt
    x0, rank = guess(A, sk.Y, b)
    assert rank == 6
    assert np.linalg.norm(A @ x0 - b) <= 1e-12 * np.linalg.norm(b)
    x, info = gmres(A, b, x0, lambda v: v.copy(), 30, 1e-10)
    assert info.iters == 0


def test_fischer_projection_special_case():
    """Fixed A, V = X, k = K: A x0 is the orthogonal projection of b onto range(B), B = A X (Sec. 4)."""
    w, g, A = _op(1)
    rs = np.random.default_rng(3)
    X = rs.standard_normal((g.n, 5))
    B = A @ X
    b = rs.standard_normal(g.n)
    x0, _ = guess(A, X, b)
    Q, _ = np.linalg.qr(B)
    assert np.allclose(A @ x0, Q @ (Q.T @ b), rtol=1e-10, atol=1e-10 * np.linalg.norm(b))


def test_forgetting_zero_gives_scaled_last_solution():
    """r = 0 keeps only x_last omega^T (Sec. 5.1: the sketch becomes rank one), so
    x0 = alpha x_last with alpha = (A x_last)^T b / ||A x_last||^2."""
    w, g, A = _op(4)
    rs = np.random.default_rng(4)
    sk = EWMASketch(g.n, 4, 0.0, 9)
    for x in rs.standard_normal((3, g.n)):
        sk.push(x)
    b = rs.standard_normal(g.n)
    x0, rank = guess(A, sk.Y, b)
    xl = x  # last pushed
    ax = A @ xl
    assert rank == 1
    assert np.allclose(x0, (ax @ b) / (ax @ ax) * xl, rtol=1e-10, atol=1e-12)


def test_span_invariance_v_equals_y_or_q():
    """span(Y) = span(Q) gives the same guess with V = Y or V = Q (Sec. 4.1.1)."""
    w, g, A = _op(6)
    rs = np.random.default_rng(5)
    Y = rs.standard_normal((g.n, 5)) @ np.diag([1, 1e-1, 1e-2, 1e-3, 1e-3])
    Q, _ = np.linalg.qr(Y)
    b = rs.standard_normal(g.n)
    x1, _ = guess(A, Y, b)
    x2, _ = guess(A, Q, b)
    assert np.linalg.norm(x1 - x2) <= 1e-9 * np.linalg.norm(x2)


def test_rank_deficient_columns_are_dropped():
    rs = np.random.default_rng(6)
    W_ = rs.standard_normal((50, 3))
    W_ = np.column_stack([W_, W_[:, 0] + W_[:, 1], W_[:, 2] * 1e-3])
    W_ /= np.linalg.norm(W_, axis=0)
    b = rs.standard_normal(50)
    z, kept = householder_lstsq_drop(W_, b)
    assert kept == [0, 1, 2]
    zz, *_ = np.linalg.lstsq(W_[:, :3], b, rcond=None)
    assert np.allclose(z, zz, rtol=1e-12)


def test_sequence_ewma_beats_previous_and_cold():
    w = W.get("tiny_17x7")
    its = {}
    for mode in ("cold", "previous", "ewma"):
        sim = Simulation.from_workload(w, guess=mode)
        tot = 0
        for s in range(w.nsys):
            ep, ec, ps = w.system(s)
            b = sim.operator(ep, ec) @ ps
            res = sim.solve(ep, ec, b)
            assert res.info.status == 0
            assert np.linalg.norm(res.x - ps) <= 1e-6 * np.linalg.norm(ps)
            tot += res.info.iters if s >= 3 else 0
        its[mode] = tot
    assert its["ewma"] < its["previous"] < its["cold"], its
