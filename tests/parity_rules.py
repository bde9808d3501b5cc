"""Decision comparison shared by the GPU parity tests.

A solve's decisions are its Arnoldi step count, restart count, true-residual checks and the
rank kept by the least-squares guess. The oracle records, per solve, how far each of its own
decisions cleared its threshold (``Result.margins``: smallest |ln(value / threshold)| over the
residual checks, the trigger tests of the Arnoldi estimate and the column-drop tests). Both
sides compute those values from operands that agree to rounding, so where every margin is at
least MARGIN (3 %) the decisions must be identical. Small grids (n <= TINY_N) must be identical
outright: their seeds are chosen so that the oracle meets no tie. On larger grids a decision
may differ only at a system where the oracle's own margin is below MARGIN, by at most two
Arnoldi steps with the same rank and restarts.
"""
import numpy as np

TINY_N = 1000
MARGIN = 3e-2
DECISIONS = ("residual", "trigger", "drop")


def margin_of(ro) -> float:
    return min((ro.margins or {}).get(k, np.inf) for k in DECISIONS)


def margins_text(ro) -> str:
    return " ".join(f"{k}={(ro.margins or {}).get(k, np.inf):.1e}" for k in DECISIONS)


def check_decisions(info, ro, n: int, label: str = "") -> bool:
    """Assert the rule above for one solve; returns True when it was a tolerated tie."""
    gd = (info.iters, info.restarts, info.checks, info.rank)
    od = (ro.info.iters, ro.info.restarts, ro.info.checks, ro.rank)
    margin = margin_of(ro)
    if n <= TINY_N:
        assert margin >= MARGIN, f"{label}: the oracle meets a tie (margin {margin:.2e}); choose another seed"
        assert gd == od, (label, gd, od)
        return False
    if gd == od:
        return False
    assert margin < MARGIN, (label, gd, od, margin)
    assert info.rank == ro.rank and info.restarts == ro.info.restarts, (label, gd, od)
    assert 0 < abs(info.iters - ro.info.iters) <= 2, (label, gd, od)
    return True
