"""Three-dimensional mixed-stage operator (test infrastructure, see package header).

Sec. 2.1 writes the sigma-transform in three dimensions: chi = x, gamma = y, sigma = (z + h)/d
with d = h + eta over the horizontal plane, and the push-forward of the gradient
grad = (d/dchi + sigma_x d/dsigma, d/dgamma + sigma_y d/dsigma, sigma_z d/dsigma) with
sigma_x = (h_chi - sigma d_chi)/d, sigma_y = (h_gamma - sigma d_gamma)/d, sigma_z = 1/d.
Sec. 3's pressure equation couples two stages through grad^(i) . grad^(i-1); in three
dimensions it gains the gamma terms of the same form as the chi terms. The paper runs its
experiments on two-dimensional vertical slices; this module is the operator on a full
(chi, gamma, sigma) grid.

Readings (the two-dimensional ones carried over, see discretization.py):

* composed first-derivative form:
  A = D_chi G_chi + diag(sigma_x^cur) D_sigma G_chi + D_gamma G_gamma
      + diag(sigma_y^cur) D_sigma G_gamma + diag(1/d^cur) D_sigma G_z,
  G_chi = D_chi + diag(sigma_x^prev) D_sigma, G_gamma = D_gamma + diag(sigma_y^prev) D_sigma,
  G_z = diag(1/d^prev) D_sigma, every D a seven-point first derivative;
* unnormalised outward normals: (-h_chi, -h_gamma, -1) at the bed, (-+1, 0, 0) at the chi
  walls, (0, -+1, 0) at the gamma walls; each direction is periodic or bounded by walls with
  one ghost column beyond each wall;
* a ghost node carries the boundary row of the one boundary it lies beyond, evaluated at the
  boundary node next to it (bed: level 1; walls: the first physical column or row); a node
  beyond two boundaries (a grid edge or corner) and every free-surface node carry identity rows;
* h and eta are extended to the ghost columns and rows by even reflection.

Layout: node (level j, row r, column c) at (j * nrow + r) * ncol + c (chi fastest, then
gamma, then sigma), level 0 the ghost level below the bed.

Pins (tests/test_oracle_operator3d.py): on fields constant in gamma each gamma row of A x is
the two-dimensional operator of discretization.py applied to that row; swapping the roles of
chi and gamma (grid, fields and vector transposed) transposes the result; sixth-order
convergence to the analytic three-dimensional composite on manufactured fields with bed and
wall rows against the analytic normal derivatives (sympy).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .fd import diff_matrix


@dataclass
class Grid3:
    nx: int
    ny: int
    nz: int
    bc_x: str  # "periodic" | "walls"
    bc_y: str
    length_x: float
    length_y: float

    def __post_init__(self):
        for bc in (self.bc_x, self.bc_y):
            if bc not in ("periodic", "walls"):
                raise ValueError(bc)
        self.per_x = self.bc_x == "periodic"
        self.per_y = self.bc_y == "periodic"
        self.ncol = self.nx - 1 if self.per_x else self.nx + 2
        self.nrow = self.ny - 1 if self.per_y else self.ny + 2
        self.nl = self.nz + 1
        self.nplane = self.ncol * self.nrow
        self.n = self.nplane * self.nl
        self.dx = self.length_x / (self.nx - 1)
        self.dy = self.length_y / (self.ny - 1)
        self.dsig = 1.0 / (self.nz - 1)
        self.sig = (np.arange(self.nl) - 1.0) * self.dsig

    def extend(self, v_phys) -> np.ndarray:
        """Plane values (nrow x ncol) including ghost rows and columns (even reflection)."""
        v = np.asarray(v_phys, dtype=np.float64)
        nyp = self.ny - 1 if self.per_y else self.ny
        nxp = self.nx - 1 if self.per_x else self.nx
        assert v.shape == (nyp, nxp), (v.shape, (nyp, nxp))
        if not self.per_x:
            v = np.concatenate((v[:, 1:2], v, v[:, -2:-1]), axis=1)
        if not self.per_y:
            v = np.concatenate((v[1:2, :], v, v[-2:-1, :]), axis=0)
        return v.copy()

    def index(self, j, r, c):
        return (np.asarray(j) * self.nrow + np.asarray(r)) * self.ncol + np.asarray(c)

    def ghost_col(self) -> np.ndarray:
        g = np.zeros(self.ncol, dtype=bool)
        if not self.per_x:
            g[0] = g[-1] = True
        return g

    def ghost_row(self) -> np.ndarray:
        g = np.zeros(self.nrow, dtype=bool)
        if not self.per_y:
            g[0] = g[-1] = True
        return g

    def row_kinds(self) -> np.ndarray:
        """Per node: 0 PDE, 1 identity, 2 bed, 3 left / 4 right chi wall, 5 front / 6 back gamma wall."""
        gc = self.ghost_col()[None, None, :]
        gr = self.ghost_row()[None, :, None]
        lev = np.arange(self.nl)[:, None, None]
        shape = (self.nl, self.nrow, self.ncol)
        kind = np.zeros(shape, dtype=np.int8)
        cidx = np.broadcast_to(np.arange(self.ncol)[None, None, :], shape)
        ridx = np.broadcast_to(np.arange(self.nrow)[:, None][None], shape)
        bed = np.broadcast_to((lev == 0) & ~gc & ~gr, shape)
        xw = np.broadcast_to((lev > 0) & (lev < self.nz) & gc & ~gr, shape)
        yw = np.broadcast_to((lev > 0) & (lev < self.nz) & gr & ~gc, shape)
        pde = np.broadcast_to((lev > 0) & (lev < self.nz) & ~gc & ~gr, shape)
        kind[...] = 1
        kind[pde] = 0
        kind[bed] = 2
        kind[xw & (cidx == 0)] = 3
        kind[xw & (cidx == self.ncol - 1)] = 4
        kind[yw & (ridx == 0)] = 5
        kind[yw & (ridx == self.nrow - 1)] = 6
        return kind.reshape(-1)

    def along_x(self, d1) -> sp.csr_matrix:
        return sp.kron(sp.identity(self.nl * self.nrow), d1, format="csr")

    def along_y(self, d1) -> sp.csr_matrix:
        return sp.kron(sp.kron(sp.identity(self.nl), d1), sp.identity(self.ncol), format="csr")

    def along_sigma(self, d1) -> sp.csr_matrix:
        return sp.kron(d1, sp.identity(self.nplane), format="csr")

    def per_column(self, v_plane) -> np.ndarray:
        return np.tile(np.asarray(v_plane, dtype=np.float64).reshape(-1), self.nl)


def surface_derivatives(grid: Grid3, width: int = 7):
    """Fixed first derivatives on the free-surface subgrid: (D_chi, D_gamma) as plane operators."""
    dxm = diff_matrix(grid.ncol, grid.dx, 1, width, grid.per_x)
    dym = diff_matrix(grid.nrow, grid.dy, 1, width, grid.per_y)
    return (sp.kron(sp.identity(grid.nrow), dxm, format="csr"),
            sp.kron(dym, sp.identity(grid.ncol), format="csr"))


def geometry3(grid: Grid3, h_phys, eta_phys, width: int = 7) -> dict:
    """Per-column d, h_chi, h_gamma, d_chi, d_gamma and per-node sigma_x, sigma_y, sigma_z (Sec. 2.1)."""
    dxp, dyp = surface_derivatives(grid, width)
    h = grid.extend(h_phys).reshape(-1)
    d = h + grid.extend(eta_phys).reshape(-1)
    if np.any(~np.isfinite(d)) or np.any(d <= 0.0):
        raise ValueError("total depth h + eta must be positive and finite")
    h_x, h_y = dxp @ h, dyp @ h
    d_x, d_y = dxp @ d, dyp @ d
    sig = grid.sig[:, None]
    sigma_x = (h_x[None, :] - sig * d_x[None, :]) / d[None, :]
    sigma_y = (h_y[None, :] - sig * d_y[None, :]) / d[None, :]
    return dict(h=h, d=d, h_x=h_x, h_y=h_y, d_x=d_x, d_y=d_y, sigma_x=sigma_x.reshape(-1),
                sigma_y=sigma_y.reshape(-1), sigma_z=grid.per_column(1.0 / d))


def _select(n: int, targets, sources) -> sp.csr_matrix:
    t = np.asarray(targets).ravel()
    s = np.asarray(sources).ravel()
    return sp.csr_matrix((np.ones(t.size), (t, s)), shape=(n, n))


def mixed_stage_operator3(grid: Grid3, h_phys, eta_prev, eta_cur, width: int = 7) -> sp.csr_matrix:
    """A(eta^(i-1), eta^(i)) = grad^(i) . grad^(i-1) on the (chi, gamma, sigma) grid with boundary rows."""
    gp = geometry3(grid, h_phys, eta_prev, width)
    gc = geometry3(grid, h_phys, eta_cur, width)
    dx = grid.along_x(diff_matrix(grid.ncol, grid.dx, 1, width, grid.per_x))
    dy = grid.along_y(diff_matrix(grid.nrow, grid.dy, 1, width, grid.per_y))
    ds = grid.along_sigma(diff_matrix(grid.nl, grid.dsig, 1, width, False))
    gx = dx + sp.diags(gp["sigma_x"]) @ ds
    gy = dy + sp.diags(gp["sigma_y"]) @ ds
    gz = sp.diags(gp["sigma_z"]) @ ds
    pde = (dx @ gx + sp.diags(gc["sigma_x"]) @ ds @ gx + dy @ gy + sp.diags(gc["sigma_y"]) @ ds @ gy
           + sp.diags(gc["sigma_z"]) @ ds @ gz)
    n, nz = grid.n, grid.nz
    kind = grid.row_kinds()
    rows = np.arange(n)
    a = _select(n, rows[kind == 0], rows[kind == 0]) @ pde
    a = a + _select(n, rows[kind == 1], rows[kind == 1])
    # bed: the ghost node below column (r, c) holds n . grad^(i-1) p at the bed node above it
    ghost = rows[kind == 2]
    bed = ghost + grid.nplane
    hx = np.zeros(n)
    hy = np.zeros(n)
    hx[bed] = gp["h_x"][bed - grid.nplane]
    hy[bed] = gp["h_y"][bed - grid.nplane]
    sel = _select(n, ghost, bed)
    a = a - sel @ (sp.diags(hx) @ gx + sp.diags(hy) @ gy + gz)
    # chi walls: -G_chi at the first physical column, +G_chi at the last
    for k, step, sign, g in ((3, 1, -1.0, gx), (4, -1, 1.0, gx),
                             (5, grid.ncol, -1.0, gy), (6, -grid.ncol, 1.0, gy)):
        t = rows[kind == k]
        if t.size:
            a = a + sign * (_select(n, t, t + step) @ g)
    a = a.tocsr()
    a.eliminate_zeros()
    return a
