"""GPU parity of the closed loop (sa_loop_*, Alg. 1) against the oracle's closed loop.

Both sides start from the same small-amplitude Airy wave on a periodic grid and step it with
LSERK45; every stage's pressure system comes from the velocity field, so each right-hand side
depends on the previous solutions (the sequence the solver is built for). After every step the
surface and both velocity components agree with the oracle's within 1e-8 of their largest
magnitude: each stage's solve reaches relative residual 1e-10 on both sides and the two solvers
take the same decisions away from ties, so the states differ by the accumulated solve
tolerance only. Arnoldi step counts are compared over the run, not per stage: each stage's
right-hand side for the dynamic pressure is rhs - A p_s, a difference of two terms far larger
than itself that each side forms with its own rounding, so the two solvers start from
right-hand sides that differ by far more than a solve's rounding and may take different steps
to the same tolerance (the states still agree to the tolerance). The mean number of steps per
solve agrees within a quarter plus one. Still water stays at rest.
"""
import sys

import numpy as np
import pytest

from oracle.closedloop import ClosedLoop as OracleLoop
from oracle.closedloop import linear_wave
from oracle.discretization import Grid
from oracle.sequence import Options, Simulation

pytestmark = pytest.mark.gpu

OPTS = dict(restart=30, rtol=1e-10, precond="mg", nu2=1, guess="ewma", k=8, r=0.9, seed=7, tau_drop=1e-7,
            coarse_max=700)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_2511_18071_amd import binding
    return binding


def _pair(B, nx, nz, waves, eta, u, w, dt, **kw):
    L = 2 * np.pi * waves
    h = np.full(nx - 1, 1.0)
    o = dict(OPTS, **kw)
    g = Grid(nx, nz, "periodic", L)
    ora = OracleLoop(g, h, eta, u, w, dt, Simulation(nx, nz, "periodic", L, h, Options(**o)))
    prob = B.Problem(nx, nz, "periodic", L, h, stream=0, **o)
    loop = B.ClosedLoop(prob, dt)
    loop.set_state(eta, u, w)
    return g, ora, prob, loop


# the loop's kernels do not depend on the solver's options; these cases run them with the
# paper's preconditioner, the range finder and the FP32 refinement path as well
CASES = [(33, 9, 1, 8, {}), (129, 17, 2, 4, {}),
         (33, 9, 1, 4, dict(precond="ilu0", guess="previous")),
         (33, 9, 1, 4, dict(guess="range", window=12)),
         (33, 9, 1, 4, dict(precision="fp32_ir")),
         (33, 9, 1, 4, dict(decay="time", decay_dtau=0.05))]


@pytest.mark.parametrize("nx,nz,waves,steps,kw", CASES)
def test_closed_loop_matches_oracle(B, nx, nz, waves, steps, kw):
    _say(f"[closed loop] {nx} x {nz}, {waves} wavelength(s), {steps} steps, {kw}")
    g = Grid(nx, nz, "periodic", 2 * np.pi * waves)
    amp, kappa = 1e-3 * waves, 1.0
    eta, u, w, om = linear_wave(g, 1.0, amp, kappa)
    dt = 2 * np.pi / om / 32
    g, ora, prob, loop = _pair(B, nx, nz, waves, eta, u, w, dt, **kw)
    gpu_its, ora_its = [], []
    for s in range(steps):
        infos = loop.step()
        k0 = len(ora.log)
        ora.step()
        e1, u1, w1 = loop.state()
        de = np.abs(e1 - ora.eta).max() / np.abs(ora.eta).max()
        du = np.abs(u1 - ora.u).max() / np.abs(ora.u).max()
        dw = np.abs(w1 - ora.w).max() / np.abs(ora.w).max()
        gi = [i.iters for i in infos]
        oi = [st["iters"] for st in ora.log[k0:]]
        _say(f"   step {s}: gpu iters {gi} oracle {oi} | d eta {de:.2e} d u {du:.2e} d w {dw:.2e}")
        assert all(i.status == 0 and i.relres <= 1e-10 for i in infos)
        assert max(de, du, dw) <= 1e-8
        gpu_its += gi
        ora_its += oi
    mg, mo = np.mean(gpu_its), np.mean(ora_its)
    _say(f"   mean steps per solve: gpu {mg:.2f} oracle {mo:.2f}")
    assert abs(mg - mo) <= 0.25 * mo + 1.0
    loop.close()
    prob.close()


def test_closed_loop_still_water(B):
    g = Grid(33, 9, "periodic", 2 * np.pi)
    z = np.zeros(g.n)
    g, ora, prob, loop = _pair(B, 33, 9, 1, np.zeros(32), z, z, 0.05)
    for _ in range(2):
        loop.step()
    e1, u1, w1 = loop.state()
    assert np.abs(u1).max() < 1e-10 and np.abs(w1).max() < 1e-10 and np.abs(e1).max() < 1e-12
    loop.close()
    prob.close()


def test_closed_loop_rejects_walls(B):
    h = np.full(33, 1.0)
    prob = B.Problem(33, 9, "walls", 1.0, h, stream=0)
    with pytest.raises(B.SawaveError) as e:
        B.ClosedLoop(prob, 0.01)
    assert e.value.code == -1
    prob.close()
