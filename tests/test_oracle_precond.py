"""Pins of the oracle's fixed preconditioners (brute-force dense solves, identities)."""
import numpy as np
import pytest

from oracle.discretization import Grid, low_order_operator
from oracle.precond import LineJacobi, VCycle, coarsen, interpolation, restriction


def _case(bc):
    if bc == "periodic":
        g = Grid(33, 7, "periodic", 2 * np.pi)
        h = 1.0 + 0.2 * np.cos(np.arange(g.ncol) * g.dx)
    else:
        g = Grid(33, 7, "walls", 3.0)
        x = np.arange(g.nx) * g.dx
        h = 0.5 - 0.3 * np.exp(-((x - 1.5) / 0.4) ** 2)
    return g, h


@pytest.mark.parametrize("bc", ["periodic", "walls"])
def test_line_jacobi_one_sweep_is_exact_column_solve(bc):
    g, h = _case(bc)
    M = low_order_operator(g, h).toarray()
    v = np.random.default_rng(1).standard_normal(g.n)
    z = LineJacobi(g, low_order_operator(g, h), nu=1, omega=1.0)(v)
    ref = np.zeros(g.n)
    for c in range(g.ncol):
        idx = np.arange(g.nl) * g.ncol + c
        ref[idx] = np.linalg.solve(M[np.ix_(idx, idx)], v[idx])
    assert np.allclose(z, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("bc", ["periodic", "walls"])
def test_coarse_max_stops_coarsening(bc):
    g, h = _case(bc)
    for cmax, expect_levels in ((g.n, 1), (g.n - 1, 2)):
        V = VCycle(g, h, coarse_max=cmax)
        assert len(V.levels) == expect_levels


@pytest.mark.parametrize("bc", ["periodic", "walls"])
def test_one_level_vcycle_is_exact_solve(bc):
    g, h = _case(bc)
    v = np.random.default_rng(2).standard_normal(g.n)
    z = VCycle(g, h, 1, 1, 0.5, max_levels=1)(v)
    ref = np.linalg.solve(low_order_operator(g, h).toarray(), v)
    assert np.allclose(z, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("bc", ["periodic", "walls"])
def test_transfer_operators(bc):
    g, h = _case(bc)
    gc, hc = coarsen(g, h)
    assert gc.ncol == (g.ncol // 2 if bc == "periodic" else (g.nx - 1) // 2 + 1 + 2)
    P, R = interpolation(g, gc), restriction(g, gc)
    # interpolation reproduces fields that are constant along x
    ones_c = np.tile(np.arange(1.0, gc.nl + 1)[:, None], (1, gc.ncol)).reshape(-1)
    ones_f = np.tile(np.arange(1.0, g.nl + 1)[:, None], (1, g.ncol)).reshape(-1)
    assert np.allclose(P @ ones_c, ones_f)
    # restriction rows sum to one (same units on both grids)
    assert np.allclose(np.asarray(R.sum(axis=1)).ravel(), 1.0)
    # interpolation is exact on fields linear in x away from the periodic seam
    if bc == "walls":
        xf = (np.arange(g.ncol) - 1) * g.dx
        xc = (np.arange(gc.ncol) - 1) * gc.dx
        lin_c = np.tile(xc, gc.nl)
        lin_f = np.tile(xf, g.nl)
        phys = np.tile(np.r_[False, np.ones(g.nx, bool), False], g.nl)
        assert np.allclose((P @ lin_c)[phys], lin_f[phys])
        # coarse depth samples are the even physical columns
        assert np.allclose(hc, h[::2])


@pytest.mark.parametrize("bc", ["periodic", "walls"])
def test_vcycle_is_linear_and_converges_as_solver(bc):
    g, h = _case(bc)
    V = VCycle(g, h, 1, 1, 0.5, coarse_max=40)
    assert len(V.levels) >= 3
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(g.n), rng.standard_normal(g.n)
    lhs = V(2.0 * u - 3.0 * v)
    rhs = 2.0 * V(u) - 3.0 * V(v)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.abs(rhs).max())
    M = low_order_operator(g, h)
    e = rng.standard_normal(g.n)
    for _ in range(20):
        e = e - V(M @ e)
        rho = np.linalg.norm(e)
        e /= rho
    assert rho < 0.6, rho
