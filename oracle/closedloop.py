"""The closed loop of Alg. 1: low-storage Runge-Kutta stepping of the velocity field and the
free surface, whose mixed-stage pressure systems are the sequence the solver is built for
(test infrastructure, see package header).

Sec. 3: at stage i the surface advances first (K_eta = alpha_i K_eta + dtau f_eta with the
kinematic condition f_eta = w - u D_chi eta at the surface), then the pressure p^(i-1) of the
mixed-stage problem grad^(i) . grad^(i-1) p = rhs is solved, where, with rho = 1,

    rhs = grad^(i) . Q,  Q = u / (beta_i dtau) + alpha_i K_u / dtau + R,
    R = F - (u . grad^(i-1)) u + (sigma / d^(i-1)) (D_tau eta) D_sigma u,

on the PDE rows, n . Q on the bed rows (n = (-h_chi, -1), the Neumann condition of the
discrete Neumann equation), 0 on the free-surface rows (p = 0); then K_u = alpha_i K_u +
dtau (R - grad^(i-1) p) and u^(i) = u^(i-1) + beta_i K_u. The scheme is the paper's with the
viscosity set to zero and gravity as the body force F = (0, -g). As in the solver the paper
builds on (Sec. 1, Sec. 2.2), the system handed to the solver is the one for the dynamic
pressure: with p_s = g d^(i-1) (1 - sigma), the hydrostatic pressure under the previous stage's
surface, A p_d = rhs - A p_s and p = p_s + p_d. Up to the solve's tolerance p is the same; the
solver sees the slowly varying dynamic part instead of a sequence dominated by the hydrostatic
one, which the guess would otherwise spend its basis on.

Readings (the paper leaves them open):

* the dynamic-pressure form above (the paper names the decomposition p = p_s + p_d and says
  its solver poses the stage problem for the dynamic pressure; p_s is taken under the surface
  at which grad^(i-1) is evaluated, so that it vanishes on the free-surface rows);
* velocities live on every node of the pressure grid, the ghost level below the bed included,
  and every node takes the same update (so that u^(i) = beta_i dtau (Q - grad^(i-1) p)
  everywhere and the discrete divergence of u^(i) at the PDE rows and n . u^(i) at the bed are
  the corresponding residuals of the pressure solve);
* D_tau eta at stage i - 1 is the kinematic right-hand side f_eta evaluated there;
* periodic in chi (the loop is built for periodic domains; the walls' boundary rows would take
  the chi component of Q in the same way);
* LSERK45 (Carpenter & Kennedy 1994) with its published coefficients, restated here.

Pins (tests/test_oracle_closedloop.py): still water stays at rest (hydrostatic pressure); after
every stage the discrete divergence of u on the PDE rows and n . u at the bed are bounded by the
pressure solve's residual; a small-amplitude progressive wave travels at the linear dispersion
relation's phase speed (omega^2 = g kappa tanh(kappa h)) and keeps its amplitude over one period;
the mean surface elevation is conserved.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import scipy.sparse as sp

from .discretization import Grid, dchi_surface, geometry
from .fd import diff_matrix

G = 9.81

# LSERK45, Carpenter & Kennedy (1994): K_i = A_i K_{i-1} + dt f(t + C_i dt, u_{i-1}); u_i = u_{i-1} + B_i K_i
LSERK_A = [Fraction(0), Fraction(-567301805773, 1357537059087), Fraction(-2404267990393, 2016746695238),
           Fraction(-3550918686646, 2091501179385), Fraction(-1275806237668, 842570457699)]
LSERK_B = [Fraction(1432997174477, 9575080441755), Fraction(5161836677717, 13612068292357),
           Fraction(1720146321549, 2090206949498), Fraction(3134564353537, 4481467310338),
           Fraction(2277821191437, 14882151754819)]
# stage times tau_n + c_i dtau
LSERK_C = [Fraction(0), Fraction(1432997174477, 9575080441755), Fraction(2526269341429, 6820363962896),
           Fraction(2006345519317, 3224310063776), Fraction(2802321613138, 2924317926251)]


class ClosedLoop:
    """State (u, w at every node; eta at the physical columns) of a periodic simulation and the
    solver (an oracle Simulation) that takes its pressure systems in sequence."""

    def __init__(self, grid: Grid, h_phys, eta, u, w, dtau: float, sim):
        if not grid.periodic:
            raise ValueError("the closed loop is built for periodic domains")
        self.grid, self.h = grid, np.asarray(h_phys, dtype=np.float64)
        self.eta = np.array(eta, dtype=np.float64)
        self.u, self.w = np.array(u, dtype=np.float64), np.array(w, dtype=np.float64)
        self.dt = float(dtau)
        self.sim = sim
        self.steps = 0  # completed steps: stage i of this step is at (steps + c_i) dtau
        self.Ku = np.zeros(grid.n)
        self.Kw = np.zeros(grid.n)
        self.Keta = np.zeros_like(self.eta)
        self.ds = grid.along_sigma(diff_matrix(grid.nl, grid.dsig, 1, 7, False))
        self.dx = grid.along_x(dchi_surface(grid))
        self.dsurf = dchi_surface(grid)
        self.sig = np.repeat(grid.sig, grid.ncol)
        self.log = []  # per stage: (relres of the solve, divergence bound check values)

    def _grad(self, eta):
        """(G_chi, G_z) = (D_chi + diag(sigma_x) D_sigma, diag(1/d) D_sigma) at a surface, and the geometry."""
        geo = geometry(self.grid, self.h, eta)
        gx = self.dx + sp.diags(geo["sigma_x"]) @ self.ds
        gz = sp.diags(geo["sigma_z"]) @ self.ds
        return geo, gx.tocsr(), gz.tocsr()

    def stage(self, i: int):
        g = self.grid
        a, b = float(LSERK_A[i]), float(LSERK_B[i])
        dt = self.dt
        u, w, eta = self.u, self.w, self.eta
        top = g.index(g.nz, np.arange(g.ncol))
        # surface: kinematic condition at stage i - 1
        f_eta = w[top] - u[top] * (self.dsurf @ eta)
        self.Keta = a * self.Keta + dt * f_eta
        eta_new = eta + b * self.Keta
        geo_p, gx_p, gz_p = self._grad(eta)
        geo_c, gx_c, gz_c = self._grad(eta_new)
        # R = F - (u . grad^(i-1)) u + (sigma / d^(i-1)) eta_t D_sigma u
        ux, uz, wx, wz = gx_p @ u, gz_p @ u, gx_p @ w, gz_p @ w
        move = self.sig * np.tile(f_eta, g.nl) * geo_p["sigma_z"]
        rx = -(u * ux + w * uz) + move * (self.ds @ u)
        rz = -G - (u * wx + w * wz) + move * (self.ds @ w)
        qx = u / (b * dt) + a * self.Ku / dt + rx
        qz = w / (b * dt) + a * self.Kw / dt + rz
        rhs = gx_c @ qx + gz_c @ qz
        kind = g.row_kinds()
        rhs[kind == 1] = 0.0
        ghost = np.nonzero(kind == 2)[0]
        bed = ghost + g.ncol
        rhs[ghost] = -geo_p["h_chi"][bed % g.ncol] * qx[bed] - qz[bed]
        # the system is posed for the dynamic pressure p_d = p - p_s, p_s = g d^(i-1) (1 - sigma)
        # the hydrostatic pressure under the previous stage's surface (zero on the surface)
        ps = G * (geo_p["d"][None, :] * (1.0 - g.sig[:, None])).reshape(-1)
        rhs = rhs - self.sim.operator(eta, eta_new) @ ps
        tau = (self.steps + float(LSERK_C[i])) * dt  # the system's time label (forgetting in time)
        res = self.sim.solve(eta, eta_new, rhs, tau=tau if self.sim.opts.decay == "time" else None)
        p = res.x + ps
        self.Ku = a * self.Ku + dt * (rx - gx_p @ p)
        self.Kw = a * self.Kw + dt * (rz - gz_p @ p)
        self.u = u + b * self.Ku
        self.w = w + b * self.Kw
        self.eta = eta_new
        # the stage's divergence at the PDE rows and n . u at the bed (each should be the solve's
        # residual times beta dtau)
        div = (gx_c @ self.u + gz_c @ self.w)[kind == 0]
        nu = -geo_p["h_chi"][bed % g.ncol] * self.u[bed] - self.w[bed]
        self.log.append(dict(relres=res.info.relres, iters=res.info.iters, rhs_norm=float(np.linalg.norm(rhs)),
                             div=float(np.abs(div).max()), nu=float(np.abs(nu).max()), scale=b * dt))
        return res

    def step(self):
        for i in range(5):
            self.stage(i)
        self.steps += 1


def linear_wave(grid: Grid, h: float, amp: float, kappa: float, t: float = 0.0):
    """Airy wave of amplitude amp and wavenumber kappa over depth h at time t: eta, u, w at the
    nodes of the sigma grid of that surface (z = sigma d - h), the ghost level included."""
    om = np.sqrt(G * kappa * np.tanh(kappa * h))
    xc = np.arange(grid.ncol) * grid.dx
    eta = amp * np.cos(kappa * xc - om * t)
    d = h + eta
    z = grid.sig[:, None] * d[None, :] - h
    ph = kappa * xc[None, :] - om * t
    u = amp * om * np.cosh(kappa * (z + h)) / np.sinh(kappa * h) * np.cos(ph)
    w = amp * om * np.sinh(kappa * (z + h)) / np.sinh(kappa * h) * np.sin(ph)
    return eta, u.reshape(-1), w.reshape(-1), om
