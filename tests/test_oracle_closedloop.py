"""Pins of the closed loop (oracle/closedloop.py): the stage formulas of Sec. 3 / Alg. 1 against
what physics and the construction fix.

* Still water stays at rest: with eta = 0 and u = 0 the right-hand side is the gravity term,
  the pressure is hydrostatic (linear in sigma, reproduced exactly by the stencils) and no
  velocity or surface motion appears.
* Incompressibility by construction: after each stage the discrete divergence grad^(i) . u^(i)
  on the PDE rows and n . u^(i) at the bed are beta_i dtau times the pressure solve's residual,
  so both stay below beta_i dtau rtol ||rhs|| (up to rounding).
* Linear waves: a small-amplitude Airy wave (kappa h = 1) travels at the phase speed of the
  linear dispersion relation omega^2 = g kappa tanh(kappa h): after a quarter period and after
  a full period the surface matches the travelled profile within 1 % of the amplitude (a wrong
  sign of gravity, of the pressure gradient or of the kinematic condition stops or reverses
  the wave, a missing factor changes its speed by far more).
* Mass: the mean surface elevation of the periodic domain is conserved.
"""
import numpy as np
import pytest

from oracle.closedloop import ClosedLoop, linear_wave
from oracle.discretization import Grid
from oracle.sequence import Options, Simulation


def _loop(nx, nz, eta, u, w, dt, rtol=1e-10, guess="ewma"):
    h, L = 1.0, 2 * np.pi
    g = Grid(nx, nz, "periodic", L)
    sim = Simulation(nx, nz, "periodic", L, np.full(nx - 1, h),
                     Options(restart=30, rtol=rtol, precond="mg", guess=guess, k=8, r=0.9))
    return g, ClosedLoop(g, np.full(nx - 1, h), eta, u, w, dt, sim)


def test_still_water_stays_at_rest():
    g = Grid(33, 9, "periodic", 2 * np.pi)
    g, lp = _loop(33, 9, np.zeros(32), np.zeros(g.n), np.zeros(g.n), 0.05)
    lp.step()
    lp.step()
    assert np.abs(lp.u).max() < 1e-10 and np.abs(lp.w).max() < 1e-10 and np.abs(lp.eta).max() < 1e-12


@pytest.fixture(scope="module")
def wave_run():
    g = Grid(33, 9, "periodic", 2 * np.pi)
    amp, kappa, h = 1e-3, 1.0, 1.0
    eta, u, w, om = linear_wave(g, h, amp, kappa)
    T = 2 * np.pi / om
    nsteps = 32
    g, lp = _loop(33, 9, eta, u, w, T / nsteps)
    snaps = {}
    for s in range(nsteps):
        lp.step()
        if s + 1 in (nsteps // 4, nsteps):
            snaps[s + 1] = lp.eta.copy()
    return g, lp, snaps, amp, kappa, h, T, nsteps, eta.mean()


def test_divergence_is_the_solve_residual(wave_run):
    g, lp, *_ = wave_run
    rtol = 1e-10
    for st in lp.log:
        assert st["relres"] <= rtol
        bound = 1.01 * st["scale"] * rtol * st["rhs_norm"]
        assert st["div"] <= bound and st["nu"] <= bound, st


def test_linear_wave_travels_at_the_dispersion_speed(wave_run):
    g, lp, snaps, amp, kappa, h, T, nsteps, _ = wave_run
    for k, t in ((nsteps // 4, T / 4), (nsteps, T)):
        ref, _, _, _ = linear_wave(g, h, amp, kappa, t=t)
        err = np.abs(snaps[k] - ref).max() / amp
        assert err < 1e-2, (k, err)
    # a quarter period moves the crest a quarter wavelength: the initial profile is far off
    ref0, _, _, _ = linear_wave(g, h, amp, kappa, t=0.0)
    assert np.abs(snaps[nsteps // 4] - ref0).max() / amp > 0.5


def test_mean_surface_is_conserved(wave_run):
    g, lp, snaps, amp, *_, mean0 = wave_run
    # the discrete surface flux is zero up to the solves' residuals (rtol 1e-10) and truncation
    assert abs(lp.eta.mean() - mean0) < 1e-6 * amp
