"""Left-preconditioned restarted GMRES (test infrastructure, see package header).

Sec. 3 solves each system with GMRES (Saad & Schultz 1986), left-preconditioned with a
fixed still-water preconditioner. Restart length, orthogonalisation, stopping rule and
restart cap are not stated in the paper; readings:

* GMRES(m) on M^-1 A x = M^-1 b, Arnoldi with classical Gram-Schmidt applied twice
  (CGS2), Givens rotations on the Hessenberg matrix;
* the decision is taken on the true residual: converged when ||b - A x|| <= rtol ||b||;
  the Arnoldi estimate |g_{j+1}| (a preconditioned residual norm) only triggers a check,
  first when it drops below rtol ||b|| ||M^-1 r0|| / ||r0||, the first cycle's preconditioned
  residual norm rescaled to the true residual's scale (so that no preconditioner application
  is spent on b alone); after a failed check the trigger threshold is lowered by the same
  rescaling with the checked candidate, to |g_{j+1}| rtol ||b|| / ||b - A x_j||, and the
  candidate is discarded;
* lucky breakdown when h_{j+1,j} <= 1e-14 ||M^-1 A v_j||: the candidate is formed, checked,
  and the cycle ends (restart from it if the check fails);
* the iteration count is the number of Arnoldi steps over all cycles; x0 already inside
  the tolerance returns after zero iterations (Sec. 5.1 observes such solves).

Every decision compares a value with a threshold; ``Info.margins`` records, per kind of
decision, the smallest |ln(value / threshold)| the solve met: 'residual' (initial accept,
every true-residual check and cycle end), 'trigger' (the Arnoldi estimate against the check
threshold, every step) and 'breakdown' (every step), so that a caller can tell a solve whose
decisions are clear-cut from one that sits at a tie.

Pins (tests/test_oracle_gmres.py): dense LU on small systems, convergence in at most p steps
for a diagonal matrix with p distinct eigenvalues, zero/one step for the identity,
restart bookkeeping on a non-normal system that needs several cycles.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

OK, NOCONV = 0, 1
BREAKDOWN_RATIO = 1e-14


@dataclass
class Info:
    iters: int = 0
    restarts: int = 0
    status: int = OK
    relres0: float = 0.0
    relres: float = 0.0
    checks: int = 0
    margins: dict = None

    def note(self, kind: str, value: float, threshold: float):
        """Record the margin of the decision value <= threshold of the given kind."""
        if self.margins is None:
            self.margins = {}
        if threshold > 0.0 and value > 0.0 and np.isfinite(value):
            m = abs(float(np.log(value / threshold)))
            self.margins[kind] = min(self.margins.get(kind, np.inf), m)


def _nrm(v) -> float:
    return float(np.sqrt(np.dot(v, v)))


def gmres(A, b, x0, minv, m: int, rtol: float, max_restarts: int = 200):
    b = np.asarray(b, dtype=np.float64)
    nb = _nrm(b)
    info = Info()
    if nb == 0.0:
        return np.zeros_like(b), info
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - A @ x
    rn = _nrm(r)
    info.relres0 = info.relres = rn / nb
    info.note("residual", rn, rtol * nb)
    if rn <= rtol * nb:
        return x, info
    trigger = None
    while True:
        z = minv(r)
        beta = _nrm(z)
        if trigger is None:
            trigger = rtol * beta * nb / rn
        V = np.zeros((m + 1, b.size))
        V[0] = z / beta
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        done = False
        jend = m
        for j in range(m):
            info.iters += 1
            w = minv(A @ V[j])
            w0 = _nrm(w)
            h1 = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h1
            h2 = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h2
            col = np.zeros(m + 1)
            col[: j + 1] = h1 + h2
            hn = _nrm(w)
            col[j + 1] = hn
            breakdown = hn <= BREAKDOWN_RATIO * w0
            info.note("breakdown", hn, BREAKDOWN_RATIO * w0)
            for i in range(j):
                t = cs[i] * col[i] + sn[i] * col[i + 1]
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1]
                col[i] = t
            den = float(np.hypot(col[j], col[j + 1]))
            cs[j], sn[j] = col[j] / den, col[j + 1] / den
            col[j], col[j + 1] = den, 0.0
            H[:, j] = col
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            info.note("trigger", abs(g[j + 1]), trigger)
            if breakdown or abs(g[j + 1]) <= trigger:
                y = _back_substitute(H[: j + 1, : j + 1], g[: j + 1])
                xc = x + V[: j + 1].T @ y
                rc = b - A @ xc
                rcn = _nrm(rc)
                info.checks += 1
                info.note("residual", rcn, rtol * nb)
                if rcn <= rtol * nb:
                    info.relres = rcn / nb
                    return xc, info
                if breakdown:
                    x, r, rn = xc, rc, rcn
                    done = True
                    break
                trigger = abs(g[j + 1]) * rtol * nb / rcn
            V[j + 1] = w / hn
        if not done:
            y = _back_substitute(H[:jend, :jend], g[:jend])
            x = x + V[:jend].T @ y
            r = b - A @ x
            rn = _nrm(r)
            info.relres = rn / nb
            info.note("residual", rn, rtol * nb)
            if rn <= rtol * nb:
                return x, info
        info.relres = rn / nb
        info.restarts += 1
        if info.restarts > max_restarts:
            info.status = NOCONV
            return x, info


def _back_substitute(R, g):
    k = g.size
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - R[i, i + 1:k] @ y[i + 1:k]) / R[i, i]
    return y
