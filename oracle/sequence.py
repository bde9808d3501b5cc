"""Per-system driver of the sequence (test infrastructure, see package header).

Alg. 1 produces one Poisson system per Runge-Kutta stage; Alg. 2 solves each one from an
initial guess taken from the subspace of previous solutions; Alg. 4 keeps that subspace as
an exponentially weighted sketch updated after every solve. Guess modes: 'cold' (x0 = 0),
'previous' (x0 = the last solution: the paper's baseline, Sec. 5.1) and 'ewma'
(x0 = Y z* once a solution has been stored and ``n_init`` solves have run; until then the
previous solution, as the paper warms the history up with the baseline, Sec. 5.1).
Every returned solution is stored, converged or not. ``precision='fp32_ir'`` solves each
system by FP64 refinement around single-precision GMRES cycles (module ``refine``).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import gmres as _gmres
from . import precond as _precond
from . import refine as _refine
from .discretization import Grid, mixed_stage_operator
from .rangefinder import RangeFinder
from .subspace import TAU_DROP, EWMASketch, guess


@dataclass
class Options:
    restart: int = 30
    max_restarts: int = 200
    rtol: float = 1e-8
    precond: str = "mg"  # none | line | mg | ilu0
    nu1: int = 1
    nu2: int = 1
    omega: float = 0.5
    max_levels: int = 32
    coarse_max: int = 700
    guess: str = "ewma"  # cold | previous | ewma | range (Alg. 3, V = X Omega)
    k: int = 8
    window: int = 16  # K, solutions kept by the range finder (guess = 'range')
    decay: str = "solves"  # 'solves' | 'time' (EWMA: forgetting exponent in time, solve(tau=...))
    decay_dtau: float = 1.0
    orthonormalize: bool = False  # range finder: V = Q
    r: float = 0.9
    seed: int = 0
    n_init: int = 0
    tau_drop: float = TAU_DROP
    precision: str = "fp64"  # fp64 | fp32_ir
    rtol_inner: float = 1e-4
    max_refine: int = 200


@dataclass
class Result:
    x: np.ndarray
    info: _gmres.Info
    rank: int = 0
    x0: np.ndarray = field(default=None, repr=False)
    margins: dict = None  # smallest decision margin per kind: 'drop' (guess) and gmres.Info's


class Simulation:
    def __init__(self, nx, nz, bc, length, h_phys, opts: Options):
        self.grid = Grid(nx, nz, bc, length)
        self.h = np.asarray(h_phys, dtype=np.float64)
        self.opts = opts
        self.minv = _precond.make(self.grid, self.h, opts.precond, opts.nu1, opts.nu2, opts.omega,
                                  opts.max_levels, opts.coarse_max)
        if opts.guess == "ewma":
            self.sketch = EWMASketch(self.grid.n, opts.k, opts.r, opts.seed,
                                     opts.decay_dtau if opts.decay == "time" else None)
        elif opts.guess == "range":
            self.sketch = RangeFinder(self.grid.n, opts.window, opts.k, opts.seed, opts.orthonormalize,
                                      opts.tau_drop)
        else:
            self.sketch = None
        self.x_prev = None
        self.solves = 0

    @classmethod
    def from_workload(cls, w, **overrides):
        kw = dict(restart=w.restart, rtol=w.rtol, precond=w.precond, nu2=getattr(w, "nu2", 1),
                  tau_drop=getattr(w, "tau_drop", TAU_DROP), k=w.k, r=w.r, seed=w.seed,
                  coarse_max=getattr(w, "coarse_max", 700))
        kw.update(overrides)
        return cls(w.nx, w.nz, w.bc, w.length, w.depth(), Options(**kw))

    def operator(self, eta_prev, eta_cur):
        return mixed_stage_operator(self.grid, self.h, eta_prev, eta_cur)

    def initial_guess(self, A, b, stats=None):
        o, n = self.opts, self.grid.n
        prev = self.x_prev if self.x_prev is not None else np.zeros(n)
        if o.guess == "cold":
            return np.zeros(n), 0
        if o.guess == "previous" or self.sketch.pushes == 0 or self.solves < o.n_init:
            return prev.copy(), 0
        V = self.sketch.basis(stats) if o.guess == "range" else self.sketch.Y
        return guess(A, V, b, o.tau_drop, stats)

    def solve(self, eta_prev, eta_cur, b, tau: float | None = None) -> Result:
        """Solve the next system of the sequence; tau is its time label (decay = 'time')."""
        if self.opts.decay == "time" and tau is None:
            raise ValueError("decay='time' needs the time label of every system")
        A = self.operator(eta_prev, eta_cur)
        stats = {}
        x0, rank = self.initial_guess(A, b, stats)
        o = self.opts
        if o.precision == "fp32_ir":
            x, info = _refine.solve(A, b, x0, self.minv, o.restart, o.rtol, o.rtol_inner, o.max_refine)
        else:
            x, info = _gmres.gmres(A, b, x0, self.minv, o.restart, o.rtol, o.max_restarts)
        if self.sketch is not None:
            if self.opts.decay == "time" and self.opts.guess == "ewma":
                self.sketch.push(x, tau)
            else:
                self.sketch.push(x)
        self.x_prev = x
        self.solves += 1
        margins = dict(getattr(info, "margins", None) or {})
        if "margin" in stats:
            margins["drop"] = stats["margin"]
        return Result(x=x, info=info, rank=rank, x0=x0, margins=margins)
