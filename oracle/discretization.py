"""Grid, sigma-transform geometry and assembled operators (test infrastructure, see package header).

Sec. 2.1: sigma = (z + h)/d with d = h + eta, and the push-forward of the gradient
grad = (d/dchi + sigma_x d/dsigma, sigma_z d/dsigma) with sigma_x = (h_chi - sigma d_chi)/d,
sigma_z = 1/d. Sec. 3: eta lives on the sigma = 1 subgrid, where D_chi is a fixed operator;
the pressure solve at stage i uses the mixed-stage operator grad^(i) . grad^(i-1)
(the discrete pressure equation), homogeneous Dirichlet p = 0 on the free surface and the
Neumann condition n . grad^(i-1) p = ... on solid boundaries, imposed through ghost nodes
so that the condition and the PDE hold together at the boundary nodes (the discrete Neumann
equation). Sec. 5.1: one ghost level below the bed; Sec. 5.2: walls with ghost nodes,
sixth-order operators.

Readings taken where the paper is silent:

* the composed first-derivative form: A = D_chi G_chi + diag(sigma_x^cur) D_sigma G_chi
  + diag(1/d^cur) D_sigma G_z, G_chi = D_chi + diag(sigma_x^prev) D_sigma,
  G_z = diag(1/d^prev) D_sigma, every D a seven-point first derivative;
* the outward normals are left unnormalised: (-h_chi, -1) at the bed, (-1, 0) / (+1, 0)
  at the left / right wall; ghost nodes that touch no boundary node (grid corners) and the
  free-surface nodes carry identity rows;
* h and eta are extended to ghost columns by even reflection.

The low-order operator M (still water, eta = 0) is the preconditioner's operator: the
direct second-order form of the sigma-transformed Laplacian,
M = D2_chi + 2 s D_chi D_sigma + (s^2 + 1/h^2) D2_sigma + s_chichi D_sigma with
s = h_chi (1 - sigma)/h and s_chichi = (1 - sigma) h_chichi/h - 2 (1 - sigma) h_chi^2/h^2,
three-point stencils, the same boundary-row types at second order.

Pins (tests/test_oracle_operator.py): sixth-order convergence of A p on manufactured
fields against the analytic mixed-stage operator (sympy), the Neumann rows against the
analytic normal derivative, the geometry against finite differences of sigma(x, z),
second-order convergence of M against the analytic Laplacian.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .fd import diff_matrix


@dataclass
class Grid:
    nx: int
    nz: int
    bc: str  # "periodic" | "walls"
    length: float

    def __post_init__(self):
        if self.bc not in ("periodic", "walls"):
            raise ValueError(self.bc)
        self.periodic = self.bc == "periodic"
        self.ncol = self.nx - 1 if self.periodic else self.nx + 2
        self.nl = self.nz + 1
        self.n = self.ncol * self.nl
        self.dx = self.length / (self.nx - 1)
        self.dsig = 1.0 / (self.nz - 1)
        self.sig = (np.arange(self.nl) - 1.0) * self.dsig  # level 0 = ghost below the bed

    def extend(self, v_phys) -> np.ndarray:
        """Column values including ghost columns (even reflection at walls)."""
        v = np.asarray(v_phys, dtype=np.float64)
        if self.periodic:
            assert v.size == self.ncol
            return v.copy()
        assert v.size == self.nx
        return np.concatenate(([v[1]], v, [v[-2]]))

    def index(self, j, c):
        return np.asarray(j) * self.ncol + np.asarray(c)

    def row_kinds(self) -> np.ndarray:
        """Per node: 0 PDE, 1 identity, 2 bed Neumann (ghost level), 3 left wall, 4 right wall."""
        kind = np.zeros((self.nl, self.ncol), dtype=np.int8)
        kind[self.nz, :] = 1
        kind[0, :] = 2
        if not self.periodic:
            kind[1:self.nz, 0] = 3
            kind[1:self.nz, -1] = 4
            kind[0, 0] = kind[0, -1] = 1
            kind[self.nz, 0] = kind[self.nz, -1] = 1
        return kind.reshape(-1)

    def along_x(self, d1: sp.spmatrix) -> sp.csr_matrix:
        return sp.kron(sp.identity(self.nl), d1, format="csr")

    def along_sigma(self, d1: sp.spmatrix) -> sp.csr_matrix:
        return sp.kron(d1, sp.identity(self.ncol), format="csr")

    def per_column(self, v) -> np.ndarray:
        return np.tile(np.asarray(v, dtype=np.float64), self.nl)


def dchi_surface(grid: Grid, width: int = 7) -> sp.csr_matrix:
    """Fixed first-derivative operator on the free-surface subgrid (ghost columns included)."""
    return diff_matrix(grid.ncol, grid.dx, 1, width, grid.periodic)


def geometry(grid: Grid, h_phys, eta_phys, width: int = 7) -> dict:
    """Per-column d, d_chi, h_chi and per-node sigma_x, sigma_z (Sec. 2.1)."""
    dchi = dchi_surface(grid, width)
    h = grid.extend(h_phys)
    d = h + grid.extend(eta_phys)
    if np.any(~np.isfinite(d)) or np.any(d <= 0.0):
        raise ValueError("total depth h + eta must be positive and finite")
    h_chi = dchi @ h
    d_chi = dchi @ d
    sig = grid.sig[:, None]
    sigma_x = (h_chi[None, :] - sig * d_chi[None, :]) / d[None, :]
    return dict(h=h, d=d, h_chi=h_chi, d_chi=d_chi, sigma_x=sigma_x.reshape(-1),
                sigma_z=grid.per_column(1.0 / d))


def _select(n: int, targets, sources) -> sp.csr_matrix:
    """Matrix E with E[t, s] = 1: moves row s of a product into row t."""
    t = np.asarray(targets).ravel()
    s = np.asarray(sources).ravel()
    return sp.csr_matrix((np.ones(t.size), (t, s)), shape=(n, n))


def _assemble(grid: Grid, pde: sp.spmatrix, gchi: sp.spmatrix, gz: sp.spmatrix, h_chi) -> sp.csr_matrix:
    """Replace rows of the PDE operator by identity / Neumann rows according to row_kinds()."""
    n, nc, nz = grid.n, grid.ncol, grid.nz
    kind = grid.row_kinds()
    rows = np.arange(n)
    a = _select(n, rows[kind == 0], rows[kind == 0]) @ pde
    a = a + _select(n, rows[kind == 1], rows[kind == 1])
    # bed: ghost node (0, c) carries n . grad p = -h_chi G_chi - G_z at the bed node (1, c)
    cols = np.nonzero(kind[:nc] == 2)[0]
    bed = grid.index(1, cols)
    hx = np.zeros(n)
    hx[bed] = h_chi[cols]
    nrm = sp.diags(hx)
    a = a - _select(n, grid.index(0, cols), bed) @ (nrm @ gchi + _select(n, bed, bed) @ gz)
    if not grid.periodic:
        lev = np.arange(1, nz)
        a = a - _select(n, grid.index(lev, 0), grid.index(lev, 1)) @ gchi
        a = a + _select(n, grid.index(lev, nc - 1), grid.index(lev, nc - 2)) @ gchi
    a = a.tocsr()
    a.eliminate_zeros()
    return a


def mixed_stage_operator(grid: Grid, h_phys, eta_prev, eta_cur, width: int = 7) -> sp.csr_matrix:
    """A(eta^(i-1), eta^(i)) = grad^(i) . grad^(i-1) with boundary rows (Sec. 3)."""
    gp = geometry(grid, h_phys, eta_prev, width)
    gc = geometry(grid, h_phys, eta_cur, width)
    dx = grid.along_x(dchi_surface(grid, width))
    ds = grid.along_sigma(diff_matrix(grid.nl, grid.dsig, 1, width, False))
    gchi = dx + sp.diags(gp["sigma_x"]) @ ds
    gz = sp.diags(gp["sigma_z"]) @ ds
    pde = dx @ gchi + sp.diags(gc["sigma_x"]) @ ds @ gchi + sp.diags(gc["sigma_z"]) @ ds @ gz
    return _assemble(grid, pde, gchi, gz, gp["h_chi"])


def low_order_operator(grid: Grid, h_phys) -> sp.csr_matrix:
    """Second-order still-water operator M (eta = 0), direct form, with the same boundary rows."""
    h = grid.extend(h_phys)
    if np.any(~np.isfinite(h)) or np.any(h <= 0.0):
        raise ValueError("still-water depth must be positive and finite")
    d1x = diff_matrix(grid.ncol, grid.dx, 1, 3, grid.periodic)
    d2x = diff_matrix(grid.ncol, grid.dx, 2, 3, grid.periodic)
    d1s = diff_matrix(grid.nl, grid.dsig, 1, 3, False)
    d2s = diff_matrix(grid.nl, grid.dsig, 2, 3, False)
    hx = d1x @ h
    hxx = d2x @ h
    one_m_sig = (1.0 - grid.sig)[:, None]
    s = (hx[None, :] * one_m_sig / h[None, :]).reshape(-1)
    sxx = (one_m_sig * hxx[None, :] / h[None, :]
           - 2.0 * one_m_sig * hx[None, :] ** 2 / h[None, :] ** 2).reshape(-1)
    inv_h = grid.per_column(1.0 / h)
    Dx, D2x = grid.along_x(d1x), grid.along_x(d2x)
    Ds, D2s = grid.along_sigma(d1s), grid.along_sigma(d2s)
    pde = D2x + 2.0 * sp.diags(s) @ Dx @ Ds + sp.diags(s * s + inv_h * inv_h) @ D2s + sp.diags(sxx) @ Ds
    gchi = Dx + sp.diags(s) @ Ds
    gz = sp.diags(inv_h) @ Ds
    return _assemble(grid, pde, gchi, gz, hx)
