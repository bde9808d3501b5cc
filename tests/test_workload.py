"""Synthetic input generator: determinism, conventions, and the LSERK45 stage times it uses."""
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_2511_18071_amd import workload as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_lserk45_is_fourth_order_on_linear_problem():
    """Apply one 2N-storage step to y' = z y symbolically: the amplification polynomial must
    match exp(z) through z^4 (Carpenter & Kennedy 1994, the paper's LSERK45, Sec. 5)."""
    # polynomial coefficients in z, exact rationals
    def add(p, q):
        n = max(len(p), len(q))
        return [(p[i] if i < len(p) else 0) + (q[i] if i < len(q) else 0) for i in range(n)]

    def scale(p, s):
        return [s * c for c in p]

    def shift(p):  # multiply by z
        return [Fraction(0)] + p

    u = [Fraction(1)]
    K = [Fraction(0)]
    for a, b in zip(W.LSERK45_A, W.LSERK45_B):
        K = add(scale(K, a), shift(u))  # K = a K + dt f(u), dt = 1, f(u) = z u
        u = add(u, scale(K, b))
    fact = [1, 1, 2, 6, 24]
    for p in range(5):
        assert abs(float(u[p]) - 1.0 / fact[p]) < 1e-11, (p, float(u[p]))
    assert abs(float(u[5]) - 1.0 / 120) > 1e-6  # not fifth order: the table is not a copy of exp


def test_lserk45_stage_times_are_consistent():
    """c_i equals the time reached by the stage input u_{i-1} of the 2N scheme for y' = 1."""
    t, K = Fraction(0), Fraction(0)
    for i, (a, b) in enumerate(zip(W.LSERK45_A, W.LSERK45_B)):
        assert abs(float(t - W.LSERK45_C[i])) < 1e-11
        K = a * K + 1
        t = t + b * K
    assert abs(float(t) - 1.0) < 1e-11


def test_battjes_limit_matches_paper_table_footnote():
    # Table 1 footnote: kh = 1.0 and H/L = 0.60 (H/L)_max = 0.0602 (Sec. 5.1)
    with open(os.path.join(GOLDEN, "battjes_table1.txt")) as f:
        kh, frac, value = [float(v) for v in f.read().split()[-3:]]
    assert abs(frac * W.battjes_max_steepness(kh) - value) / value < 0.02


@pytest.mark.parametrize("name", ["periodic_65x9", "bar_513x17", "tiny_17x7", "bar_65x9"])
def test_workload_shapes_and_determinism(name):
    w1, w2 = W.get(name), W.get(name)
    e1 = w1.system(7)
    e2 = w2.system(7)
    for a, b in zip(e1, e2):
        assert np.array_equal(a, b)
    ep, ec, ps = e1
    assert ep.shape == (w1.nphys,) and ec.shape == (w1.nphys,)
    assert ps.shape == (w1.n,)
    assert np.all(w1.depth() + ep > 0)
    # the manufactured pressure vanishes on the free surface (sigma = 1)
    assert np.allclose(ps.reshape(w1.nl, w1.ncol)[w1.nz], 0.0, atol=1e-15)
    tp, tc = w1.stage_times(7)
    assert tc > tp


def test_stream_steepness_scaling():
    w = W.get("periodic_65x9")
    x = np.linspace(0, w.length, 4096, endpoint=False)
    eta = w.surface(0.0, x)
    lam = 2 * np.pi / w.params["kappa0"]
    assert abs((eta.max() - eta.min()) / lam - 0.05) < 1e-3


def test_serving_mix_is_seeded():
    a = W.serving_mix(8, seed=5, nsys=3)
    b = W.serving_mix(8, seed=5, nsys=3)
    assert [(w.nx, w.nz, w.bc, w.k) for w in a] == [(w.nx, w.nz, w.bc, w.k) for w in b]
    for w in a:
        assert W.hierarchy_fits(w.nx, w.nz, w.bc, dense_max=1024) and 257 <= w.nx <= 8193
        assert w.nz in (9, 17, 33) and 8 <= w.k <= 16


def test_serving_mix_grid_sizes_stay_near_the_uniform_draw():
    """nx is the uniform draw moved to the nearest size whose hierarchy fits: within a few
    per cent, and the draw itself when it fits."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        nx_u = float(rng.uniform(257, 8193))
        nz = int(rng.choice((9, 17, 33)))
        bc = "periodic" if rng.uniform() < 0.5 else "walls"
        nx = W.nearest_fitting_nx(nx_u, nz, bc)
        assert W.hierarchy_fits(nx, nz, bc, dense_max=1024)
        assert abs(nx - nx_u) <= 0.04 * nx_u
        if W.hierarchy_fits(int(round(nx_u)), nz, bc, dense_max=1024):
            assert nx == int(round(nx_u))


def test_hierarchy_fits_rule():
    # periodic nz = 33 (34 levels): 4096 columns halve to 16 (544 unknowns); 4095 is odd
    assert W.hierarchy_fits(4097, 33, "periodic") and not W.hierarchy_fits(4096, 33, "periodic")
    # 1984 = 31 * 64 columns end at 31 x 34 = 1054 unknowns: over the serving mix's 1024, within
    # the library's 4096; 4064 = 127 * 32 at 127 x 34 = 4318 over both
    assert not W.hierarchy_fits(1985, 33, "periodic", dense_max=1024) and W.hierarchy_fits(1985, 33, "periodic")
    assert not W.hierarchy_fits(4065, 33, "periodic") and W.hierarchy_fits(961, 33, "periodic", dense_max=1024)
    # walls: nx - 1 must halve; 4097 points halve down, 4098 do not
    assert W.hierarchy_fits(4097, 9, "walls") and not W.hierarchy_fits(4098, 9, "walls")
