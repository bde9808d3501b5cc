"""Pins of the three-dimensional mixed-stage operator (oracle/operator3d.py).

Three independent checks, so that a dropped term, a swapped stage, a sign slip or an
exchanged chi/gamma index fails one of them:

* fields constant in gamma: every gamma row of A x is the two-dimensional operator of
  oracle/discretization.py (itself pinned by sixth-order convergence) applied to that row;
* the chi and gamma directions play the same role: swapping them (grid sizes, boundary
  conditions, lengths, the fields and the vector transposed) transposes A x;
* sixth-order convergence to the analytic composite grad^(i) . grad^(i-1) p in three
  dimensions (Sec. 2.1 push-forward, Sec. 3 mixed-stage operator), bed rows to
  n . grad^(i-1) p with n = (-h_chi, -h_gamma, -1), wall rows to -+ the chi or gamma
  component of grad^(i-1) p, on fields that vary in both horizontal directions.
"""
import numpy as np
import pytest
import sympy as sym

from oracle.discretization import Grid, mixed_stage_operator
from oracle.operator3d import Grid3, geometry3, mixed_stage_operator3

X, Y, S = sym.symbols("chi gamma sigma", real=True)


def _rng_fields(g3, seed):
    rng = np.random.default_rng(seed)
    nyp = g3.ny - 1 if g3.per_y else g3.ny
    nxp = g3.nx - 1 if g3.per_x else g3.nx
    return rng, nyp, nxp


@pytest.mark.parametrize("bc", ["periodic", "walls"])
def test_constant_in_gamma_reduces_to_two_dimensions(bc):
    g3 = Grid3(21, 9, 9, bc, "periodic", 3.0, 2.0)
    g2 = Grid(21, 9, bc, 3.0)
    rng, nyp, nxp = _rng_fields(g3, 3)
    h1 = 0.6 + 0.1 * rng.random(nxp)
    ep1 = 0.05 * rng.standard_normal(nxp)
    ec1 = 0.05 * rng.standard_normal(nxp)
    x2 = rng.standard_normal(g2.n)
    tile = lambda v: np.tile(v, (nyp, 1))
    A3 = mixed_stage_operator3(g3, tile(h1), tile(ep1), tile(ec1))
    x3 = np.repeat(x2.reshape(g2.nl, 1, g2.ncol), g3.nrow, axis=1).reshape(-1)
    y3 = (A3 @ x3).reshape(g3.nl, g3.nrow, g3.ncol)
    y2 = (mixed_stage_operator(g2, h1, ep1, ec1) @ x2).reshape(g2.nl, g2.ncol)
    scale = np.abs(y2).max()
    for r in range(g3.nrow):
        assert np.abs(y3[:, r, :] - y2).max() <= 1e-12 * scale


@pytest.mark.parametrize("bcx,bcy", [("walls", "periodic"), ("periodic", "walls"), ("walls", "walls")])
def test_chi_and_gamma_are_interchangeable(bcx, bcy):
    g = Grid3(13, 11, 8, bcx, bcy, 2.0, 1.5)
    gt = Grid3(11, 13, 8, bcy, bcx, 1.5, 2.0)
    rng, nyp, nxp = _rng_fields(g, 7)
    h = 0.5 + 0.2 * rng.random((nyp, nxp))
    ep = 0.04 * rng.standard_normal((nyp, nxp))
    ec = 0.04 * rng.standard_normal((nyp, nxp))
    x = rng.standard_normal(g.n)
    y = (mixed_stage_operator3(g, h, ep, ec) @ x).reshape(g.nl, g.nrow, g.ncol)
    xt = x.reshape(g.nl, g.nrow, g.ncol).transpose(0, 2, 1).reshape(-1)
    yt = (mixed_stage_operator3(gt, h.T, ep.T, ec.T) @ xt).reshape(gt.nl, gt.nrow, gt.ncol)
    assert np.abs(yt.transpose(0, 2, 1) - y).max() <= 1e-12 * np.abs(y).max()


def _analytic(bcx, bcy):
    """Manufactured h, eta_prev, eta_cur, p with the exact operator, normal derivatives and the
    chi/gamma components of grad^(i-1) p. Wall directions use fields even about both walls."""
    if bcx == "periodic":
        Lx, cx = 2 * sym.pi, X
    else:
        Lx, cx = sym.Integer(1), sym.pi * X
    if bcy == "periodic":
        Ly, cy = 2 * sym.pi, Y
    else:
        Ly, cy = sym.Integer(1), sym.pi * Y
    h = sym.Rational(1, 2) + sym.Rational(1, 10) * sym.cos(cx) + sym.Rational(1, 20) * sym.cos(cy)
    ep = sym.Rational(3, 100) * sym.cos(cx + 0) * sym.cos(cy) + sym.Rational(1, 100) * sym.cos(2 * cy)
    ec = sym.Rational(33, 1000) * sym.cos(cx) * sym.cos(cy) + sym.Rational(1, 100) * sym.cos(2 * cx)
    # periodic directions take 2 pi-periodic fields; wall directions any smooth field
    ax = 1 if bcx == "periodic" else sym.pi / 2
    ay = 1 if bcy == "periodic" else sym.pi / 3
    P = (sym.cos(ax * X + ay * Y + sym.Rational(1, 3)) * sym.exp(sym.Rational(7, 10) * S)
         + sym.sin(2 * ax * X) * sym.cos(ay * Y) * S ** 2)
    dp, dc = h + ep, h + ec
    hx, hy = sym.diff(h, X), sym.diff(h, Y)
    sxp = (hx - S * sym.diff(dp, X)) / dp
    syp = (hy - S * sym.diff(dp, Y)) / dp
    sxc = (hx - S * sym.diff(dc, X)) / dc
    syc = (hy - S * sym.diff(dc, Y)) / dc
    Fx = sym.diff(P, X) + sxp * sym.diff(P, S)
    Fy = sym.diff(P, Y) + syp * sym.diff(P, S)
    Fz = sym.diff(P, S) / dp
    y = (sym.diff(Fx, X) + sxc * sym.diff(Fx, S) + sym.diff(Fy, Y) + syc * sym.diff(Fy, S)
         + sym.diff(Fz, S) / dc)
    bed = -hx * Fx - hy * Fy - Fz
    f = lambda e: sym.lambdify((X, Y, S), e, "numpy")
    return float(Lx), float(Ly), dict(h=f(h), ep=f(ep), ec=f(ec), P=f(P), y=f(y), bed=f(bed), Fx=f(Fx), Fy=f(Fy))


def _coords(g):
    xc = np.arange(g.ncol) * g.dx if g.per_x else (np.arange(g.ncol) - 1) * g.dx
    yc = np.arange(g.nrow) * g.dy if g.per_y else (np.arange(g.nrow) - 1) * g.dy
    return xc, yc


def _ev(fn, *a):
    return np.broadcast_to(fn(*a), np.broadcast(*a).shape).astype(float)


@pytest.mark.parametrize("bcx,bcy", [("periodic", "periodic"), ("walls", "walls")])
def test_sixth_order_against_the_analytic_operator(bcx, bcy):
    Lx, Ly, an = _analytic(bcx, bcy)
    e_int, e_bed, e_wall = [], [], []
    for nx, nz in [(17, 13), (33, 25), (65, 49)]:
        g = Grid3(nx, nx, nz, bcx, bcy, Lx, Ly)
        xc, yc = _coords(g)
        xp = xc if g.per_x else xc[1:-1]
        yp = yc if g.per_y else yc[1:-1]
        YP, XP = np.meshgrid(yp, xp, indexing="ij")
        h = _ev(an["h"], XP, YP, 0 * XP)
        ep = _ev(an["ep"], XP, YP, 0 * XP)
        ec = _ev(an["ec"], XP, YP, 0 * XP)
        SS, YY, XX = np.meshgrid(g.sig, yc, xc, indexing="ij")
        p = _ev(an["P"], XX, YY, SS).reshape(-1)
        y = (mixed_stage_operator3(g, h, ep, ec) @ p).reshape(g.nl, g.nrow, g.ncol)
        kind = g.row_kinds().reshape(g.nl, g.nrow, g.ncol)
        yex = _ev(an["y"], XX, YY, SS)
        interior = kind == 0
        # rows whose outer and inner stencils are both centred: 6 nodes from any boundary
        interior[:6] = interior[-6:] = False
        if not g.per_x:
            interior[:, :, :6] = interior[:, :, -6:] = False
        if not g.per_y:
            interior[:, :6, :] = interior[:, -6:, :] = False
        e_int.append(np.abs(y - yex)[interior].max())
        bed = kind[0] == 2
        bed_ex = _ev(an["bed"], XX[1], YY[1], 0 * XX[1])
        e_bed.append(np.abs(y[0] - bed_ex)[bed].max())
        if bcx == "walls":
            lev = np.arange(1, g.nz)
            rows = np.arange(1, g.nrow - 1)
            LL, RR = np.meshgrid(lev, rows, indexing="ij")
            sig, yv = g.sig[LL], yc[RR]
            left = -_ev(an["Fx"], 0 * sig, yv, sig)
            right = _ev(an["Fx"], Lx + 0 * sig, yv, sig)
            front = -_ev(an["Fy"], xc[RR], 0 * sig, sig)
            back = _ev(an["Fy"], xc[RR], Ly + 0 * sig, sig)
            e_wall.append(max(np.abs(y[LL, RR, 0] - left).max(), np.abs(y[LL, RR, -1] - right).max(),
                              np.abs(y[LL, 0, RR] - front).max(), np.abs(y[LL, -1, RR] - back).max()))
    rate = lambda e: np.log2(np.array(e[:-1]) / np.array(e[1:]))
    # the coarsest walls grid (17 points) is still pre-asymptotic: 4.9 there, 6.0 after
    assert np.all(rate(e_int) > 4.5) and rate(e_int)[-1] > 5.5, (e_int, rate(e_int))
    assert np.all(rate(e_bed) > 4.5), (e_bed, rate(e_bed))
    if bcx == "walls":
        assert np.all(rate(e_wall) > 4.5), (e_wall, rate(e_wall))


def test_geometry_matches_finite_differences_of_sigma():
    """sigma_x and sigma_y of Sec. 2.1 against centred differences of sigma(x, y, z) at fixed z."""
    g = Grid3(65, 49, 9, "periodic", "periodic", 2 * np.pi, 2 * np.pi)
    xc, yc = _coords(g)
    YP, XP = np.meshgrid(yc, xc, indexing="ij")
    hf = lambda x, y: 1.0 + 0.1 * np.cos(x) + 0.05 * np.sin(y)
    ef = lambda x, y: 0.05 * np.sin(x + 0.3) * np.cos(y)
    geo = geometry3(g, hf(XP, YP), ef(XP, YP))
    sig = g.sig[:, None, None]
    z = sig * (hf(XP, YP) + ef(XP, YP)) - hf(XP, YP)
    sigma = lambda x, y: (z + hf(x, y)) / (hf(x, y) + ef(x, y))
    e = 1e-5
    sx = (sigma(XP + e, YP) - sigma(XP - e, YP)) / (2 * e)
    sy = (sigma(XP, YP + e) - sigma(XP, YP - e)) / (2 * e)
    assert np.abs(geo["sigma_x"] - sx.reshape(-1)).max() < 1e-5
    assert np.abs(geo["sigma_y"] - sy.reshape(-1)).max() < 1e-5


def test_boundary_row_kinds():
    g = Grid3(9, 8, 7, "walls", "walls", 1.0, 1.0)
    kind = g.row_kinds().reshape(g.nl, g.nrow, g.ncol)
    assert np.all(kind[g.nz] == 1)
    assert np.all(kind[0, 1:-1, 1:-1] == 2) and np.all(kind[0, 0, :] == 1) and np.all(kind[0, :, 0] == 1)
    assert np.all(kind[1:g.nz, 1:-1, 0] == 3) and np.all(kind[1:g.nz, 1:-1, -1] == 4)
    assert np.all(kind[1:g.nz, 0, 1:-1] == 5) and np.all(kind[1:g.nz, -1, 1:-1] == 6)
    assert np.all(kind[1:g.nz, 0, 0] == 1) and np.all(kind[1:g.nz, -1, -1] == 1)
    A = mixed_stage_operator3(g, np.full((g.ny, g.nx), 0.5), np.zeros((g.ny, g.nx)), np.zeros((g.ny, g.nx)))
    ident = np.nonzero(kind.reshape(-1) == 1)[0]
    sub = A[ident][:, ident].toarray()
    assert np.allclose(sub, np.eye(ident.size)) and A[ident].nnz == ident.size
