"""Pins of the oracle's geometry and operators against analytic fields.

The mixed-stage operator of Sec. 3 is grad^(i) . grad^(i-1) with the push-forward of
Sec. 2.1, so for smooth fields the discrete A p must converge to the analytic composite
d/dchi F_chi + sigma_x^cur dF_chi/dsigma + (1/d^cur) dF_z/dsigma, where
F_chi = P_chi + sigma_x^prev P_sigma and F_z = P_sigma / d^prev, at sixth order in the
interior. Boundary rows converge to the analytic normal derivative n . grad^(i-1) p with
n = (-h_chi, -1) at the bed and (-+1, 0) at the walls. The low-order still-water operator
converges to the analytic Laplacian at second order. A swapped stage, a dropped
coefficient or a wrong sign changes the limit and fails these tests.
"""
import numpy as np
import pytest
import sympy as sym

from oracle.discretization import Grid, geometry, low_order_operator, mixed_stage_operator

X, S = sym.symbols("chi sigma", real=True)


def _fields(bc):
    if bc == "periodic":
        L = 2 * sym.pi
        h = 1 + sym.Rational(1, 10) * sym.cos(X)
        ep = sym.Rational(1, 20) * sym.sin(X + sym.Rational(3, 10)) + sym.Rational(1, 50) * sym.cos(2 * X)
        ec = sym.Rational(1, 20) * sym.sin(X + sym.Rational(7, 20)) + sym.Rational(21, 1000) * sym.cos(2 * X + sym.Rational(1, 10))
        P = sym.cos(X + sym.Rational(1, 2)) * sym.exp(sym.Rational(7, 10) * S) + sym.Rational(3, 10) * sym.sin(2 * X) * S ** 2
    else:  # walls at 0 and L: h and eta even about both walls (the solver reflects them)
        L = sym.Integer(1)
        h = sym.Rational(1, 2) + sym.Rational(1, 10) * sym.cos(sym.pi * X)
        ep = sym.Rational(3, 100) * sym.cos(2 * sym.pi * X) + sym.Rational(1, 100) * sym.cos(sym.pi * X)
        ec = sym.Rational(3, 100) * sym.cos(2 * sym.pi * X + 0) * sym.Rational(11, 10) + sym.Rational(1, 100) * sym.cos(3 * sym.pi * X)
        P = sym.cos(sym.pi * X / 2 + sym.Rational(1, 3)) * sym.exp(sym.Rational(7, 10) * S) + X ** 3 * S
    return L, h, ep, ec, P


def _analytic(bc):
    L, h, ep, ec, P = _fields(bc)
    dp, dc = h + ep, h + ec
    hx = sym.diff(h, X)
    sxp = (hx - S * sym.diff(dp, X)) / dp
    sxc = (hx - S * sym.diff(dc, X)) / dc
    Fx = sym.diff(P, X) + sxp * sym.diff(P, S)
    Fz = sym.diff(P, S) / dp
    y = sym.diff(Fx, X) + sxc * sym.diff(Fx, S) + sym.diff(Fz, S) / dc
    bed = -hx * Fx - Fz
    f = lambda e: sym.lambdify((X, S), e, "numpy")
    return float(L), dict(h=f(h), ep=f(ep), ec=f(ec), P=f(P), y=f(y), bed=f(bed), Fx=f(Fx))


def _grid_fields(bc, nx, nz, an, L):
    g = Grid(nx, nz, bc, L)
    if bc == "periodic":
        xc = np.arange(g.ncol) * g.dx
        xphys = xc
    else:
        xc = (np.arange(g.ncol) - 1) * g.dx
        xphys = xc[1:-1]
    XX, SS = np.meshgrid(xc, g.sig)
    ev = lambda fn, *a: np.broadcast_to(fn(*a), np.broadcast(*a).shape).astype(float)
    h = ev(an["h"], xphys, 0 * xphys)
    ep = ev(an["ep"], xphys, 0 * xphys)
    ec = ev(an["ec"], xphys, 0 * xphys)
    p = ev(an["P"], XX, SS).reshape(-1)
    return g, h, ep, ec, p, XX, SS


@pytest.mark.parametrize("bc", ["periodic", "walls"])
def test_mixed_stage_operator_sixth_order(bc):
    L, an = _analytic(bc)
    e_int, e_all, e_bed, e_wall = [], [], [], []
    for nx, nz in [(33, 17), (65, 33), (129, 65)]:
        g, h, ep, ec, p, XX, SS = _grid_fields(bc, nx, nz, an, L)
        A = mixed_stage_operator(g, h, ep, ec)
        y = (A @ p).reshape(g.nl, g.ncol)
        kind = g.row_kinds().reshape(g.nl, g.ncol)
        yex = np.broadcast_to(an["y"](XX, SS), XX.shape)
        pde = kind == 0
        interior = pde.copy()
        # rows whose outer and inner stencils are both centred: 7 nodes from any boundary
        interior[:7] = interior[-7:] = False
        if bc == "walls":
            interior[:, :7] = interior[:, -7:] = False
        e_all.append(np.abs(y - yex)[pde].max())
        e_int.append(np.abs(y - yex)[interior].max())
        # bed rows: ghost level 0 holds n . grad^(i-1) p at the bed (sigma = 0)
        cols = np.nonzero(kind[0] == 2)[0]
        bed_ex = np.broadcast_to(an["bed"](XX[1, cols], 0 * XX[1, cols]), cols.shape)
        e_bed.append(np.abs(y[0, cols] - bed_ex).max())
        if bc == "walls":
            lev = np.arange(1, g.nz)
            left = -np.broadcast_to(an["Fx"](0 * g.sig[lev], g.sig[lev]), lev.shape)
            right = np.broadcast_to(an["Fx"](L + 0 * g.sig[lev], g.sig[lev]), lev.shape)
            e_wall.append(max(np.abs(y[lev, 0] - left).max(), np.abs(y[lev, -1] - right).max()))
    rate = lambda e: np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(rate(e_int) > 5.0) and rate(e_int)[-1] > 5.5, (e_int, rate(e_int))
    assert np.all(rate(e_all) > 4.5), (e_all, rate(e_all))
    assert np.all(rate(e_bed) > 5.0), (e_bed, rate(e_bed))
    assert e_int[-1] < 1e-6
    if bc == "walls":
        assert np.all(rate(e_wall) > 5.0), (e_wall, rate(e_wall))


def test_stage_order_matters():
    """Swapping prev and cur changes A by O(1) in the discrete sense (the operator is mixed)."""
    L, an = _analytic("periodic")
    g, h, ep, ec, p, XX, SS = _grid_fields("periodic", 33, 17, an, L)
    a1 = mixed_stage_operator(g, h, ep, ec) @ p
    a2 = mixed_stage_operator(g, h, ec, ep) @ p
    assert np.abs(a1 - a2).max() > 1e-3
    # same-stage operator is the sigma-transformed Laplacian: symmetric in prev/cur by construction
    a3 = mixed_stage_operator(g, h, ep, ep) @ p
    assert np.abs(a3 - a1).max() > 1e-4


def test_identity_rows_and_surface():
    g = Grid(17, 7, "walls", 1.0)
    h = np.full(g.nx, 0.5)
    A = mixed_stage_operator(g, h, 0 * h, 0 * h).tocsr()
    kind = g.row_kinds()
    for r in np.nonzero(kind == 1)[0]:
        row = A.getrow(r)
        assert row.nnz == 1 and row.indices[0] == r and row.data[0] == 1.0


def test_geometry_matches_finite_differences_of_sigma():
    """sigma_x = (h_chi - sigma d_chi)/d (Sec. 2.1) against a centred difference of
    sigma(x, z) = (z + h(x))/(h(x) + eta(x)) at fixed z."""
    g = Grid(129, 9, "periodic", 2 * np.pi)
    x = np.arange(g.ncol) * g.dx
    hf = lambda x: 1.0 + 0.1 * np.cos(x)
    ef = lambda x: 0.05 * np.sin(x + 0.3)
    geo = geometry(g, hf(x), ef(x))
    sx = geo["sigma_x"].reshape(g.nl, g.ncol)
    eps = 1e-5
    for j in (1, 4, 8):
        z = g.sig[j] * (hf(x) + ef(x)) - hf(x)  # the physical height of node (j, c)
        sig = lambda xx: (z + hf(xx)) / (hf(xx) + ef(xx))
        fdx = (sig(x + eps) - sig(x - eps)) / (2 * eps)
        assert np.abs(sx[j] - fdx).max() < 1e-8
    assert np.allclose(geo["sigma_z"].reshape(g.nl, g.ncol)[3], 1.0 / (hf(x) + ef(x)))


def test_low_order_operator_second_order_laplacian():
    """M (still water, direct form) -> the physical Laplacian of p(x, z) at second order."""
    xs, zs = sym.symbols("x z", real=True)
    h = 1 + sym.Rational(1, 10) * sym.cos(xs)
    p = sym.cos(xs + sym.Rational(1, 2)) * sym.exp(zs) + zs ** 3 * sym.sin(xs)
    lap = sym.diff(p, xs, 2) + sym.diff(p, zs, 2)
    hf = sym.lambdify(xs, h, "numpy")
    pf = sym.lambdify((xs, zs), p, "numpy")
    lf = sym.lambdify((xs, zs), lap, "numpy")
    errs = []
    for nx, nz in [(33, 17), (65, 33), (129, 65)]:
        g = Grid(nx, nz, "periodic", 2 * np.pi)
        x = np.arange(g.ncol) * g.dx
        hh = hf(x)
        XX, SS = np.meshgrid(x, g.sig)
        Z = SS * hf(XX) - hf(XX)
        M = low_order_operator(g, hh)
        y = (M @ pf(XX, Z).reshape(-1)).reshape(g.nl, g.ncol)
        pde = g.row_kinds().reshape(g.nl, g.ncol) == 0
        errs.append(np.abs(y - lf(XX, Z))[pde].max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), (errs, rates)


def test_rejects_nonpositive_depth():
    g = Grid(17, 7, "periodic", 1.0)
    h = np.full(g.ncol, 0.1)
    with pytest.raises(ValueError):
        mixed_stage_operator(g, h, -0.2 + 0 * h, 0 * h)


@pytest.mark.parametrize("bc", ["periodic", "walls"])
def test_low_order_operator_boundary_rows_second_order(bc):
    """M's bed and wall rows (still water, d = h) converge at second order to the analytic
    normal derivative of the previous-stage gradient at eta = 0: -h_chi F_chi - F_z at the
    bed, -+F_chi at the left / right wall, with F_chi = P_chi + sigma_x P_sigma,
    sigma_x = h_chi (1 - sigma)/h and F_z = P_sigma / h (Sec. 3 discrete Neumann equation
    with the still-water geometry); its PDE rows converge to the sigma-transformed Laplacian
    on the same grid. A flipped sign, a dropped h_chi or 1/h, or a wall row taken at the
    wrong column changes the limit."""
    L, h, _, _, P = _fields(bc)
    hx = sym.diff(h, X)
    sx = hx * (1 - S) / h
    Fx = sym.diff(P, X) + sx * sym.diff(P, S)
    Fz = sym.diff(P, S) / h
    y = sym.diff(Fx, X) + sx * sym.diff(Fx, S) + sym.diff(Fz, S) / h
    f = lambda e: sym.lambdify((X, S), e, "numpy")
    an = dict(h=f(h), ep=f(0 * X), ec=f(0 * X), P=f(P), y=f(y), bed=f(-hx * Fx - Fz), Fx=f(Fx))
    Lf = float(L)
    e_pde, e_bed, e_wall = [], [], []
    for nx, nz in [(33, 17), (65, 33), (129, 65)]:
        g, hh, _, _, p, XX, SS = _grid_fields(bc, nx, nz, an, Lf)
        yv = (low_order_operator(g, hh) @ p).reshape(g.nl, g.ncol)
        kind = g.row_kinds().reshape(g.nl, g.ncol)
        yex = np.broadcast_to(an["y"](XX, SS), XX.shape)
        e_pde.append(np.abs(yv - yex)[kind == 0].max())
        cols = np.nonzero(kind[0] == 2)[0]
        bed_ex = np.broadcast_to(an["bed"](XX[1, cols], 0 * XX[1, cols]), cols.shape)
        e_bed.append(np.abs(yv[0, cols] - bed_ex).max())
        if bc == "walls":
            lev = np.arange(1, g.nz)
            left = -np.broadcast_to(an["Fx"](0 * g.sig[lev], g.sig[lev]), lev.shape)
            right = np.broadcast_to(an["Fx"](Lf + 0 * g.sig[lev], g.sig[lev]), lev.shape)
            e_wall.append(max(np.abs(yv[lev, 0] - left).max(), np.abs(yv[lev, -1] - right).max()))
    rate = lambda e: np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(rate(e_pde) > 1.8), (e_pde, rate(e_pde))
    assert np.all(rate(e_bed) > 1.8), (e_bed, rate(e_bed))
    if bc == "walls":
        assert np.all(rate(e_wall) > 1.8), (e_wall, rate(e_wall))


def test_low_order_boundary_pin_catches_planted_mistakes(monkeypatch):
    """The boundary pin above fails for a plausible mistake planted in the oracle: the bed
    row without its h_chi term (planted by zeroing h_chi in the assembly of boundary rows)."""
    import oracle.discretization as D

    orig = D._assemble

    def planted(grid, pde, gchi, gz, h_chi):
        return orig(grid, pde, gchi, gz, 0.0 * np.asarray(h_chi))

    monkeypatch.setattr(D, "_assemble", planted)
    with pytest.raises(AssertionError):
        test_low_order_operator_boundary_rows_second_order("walls")
