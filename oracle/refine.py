"""Mixed-precision iterative refinement (test infrastructure, see package header).

The paper solves every system in double precision (Sec. 5). The refinement path keeps its
problem and its stopping rule (the true relative residual, the reading in ``gmres``) and
computes the corrections in single precision: iterative refinement (Wilkinson 1963, Moler
1967) with a GMRES cycle as the inner solver (GMRES-based refinement, Carson & Higham, SIAM
J. Sci. Comput. 2018), whose candidates are checked on the FP64 residual the way ``gmres``
checks its own. Written from that definition:

    r = b - A x0, stop at once if ||r|| <= rtol ||b||                (FP64)
    repeat (one correction per pass; NOCONV after max_refine):
        s = fl32(r / ||r||), g_0 = ||M^-1 s|| (FP32 V-cycle); at the first pass
        trigger = rtol ||b|| g_0 (the trigger of ``gmres`` in this cycle's units); a GMRES cycle of at most m steps on A d = s in which every
        operator and preconditioner application and every basis vector is rounded to
        FP32 (Gram-Schmidt sums, Hessenberg, Givens FP64); after step j with estimate
        e = ||r|| |g_{j+1}|:
          * floor: |g_{j+1}| <= rtol_inner |g_0| or h_{j+1,j} <= 1e-7 ||w|| (FP32 resolution
            reached), or e <= trigger: form x_c = x + ||r|| V y and r_c = b - A x_c (FP64);
            converged if ||r_c|| <= rtol ||b||; at the floor x, r <- x_c, r_c and the next
            correction starts; otherwise trigger <- e rtol ||b|| / ||r_c|| and the cycle goes on
        after m steps: x <- x + ||r|| V y, r <- b - A x (FP64), converged or next correction

``inner`` selects the rounding of the inner cycle: ``np.float32`` (the path) or
``np.float64`` (no rounding, for the pins).

Pins (tests/test_oracle_refine.py): with inner FP64 and the floor below reach, one cycle
solves a small system to dense-LU accuracy; with the trigger never firing the residual
contracts by at least the inner tolerance per correction on a well-conditioned system
(Carson & Higham's convergence condition); with inner FP32 the result reaches rtol = 1e-10
and agrees with the dense-LU solution to kappa * rtol.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

OK, NOCONV = 0, 1


@dataclass
class Info:
    iters: int = 0
    refinements: int = 0
    status: int = OK
    checks: int = 0
    relres0: float = 0.0
    relres: float = 0.0
    history: list = None  # relative residual after each correction


def _nrm(v) -> float:
    v = np.asarray(v, dtype=np.float64)
    return float(np.sqrt(np.dot(v, v)))


def solve(A, b, x0, minv, m: int, rtol: float, rtol_inner: float = 1e-4, max_refine: int = 200,
          inner=np.float32, use_trigger: bool = True):
    """x with ||b - A x|| <= rtol ||b|| by refinement around single-precision GMRES cycles."""
    b = np.asarray(b, dtype=np.float64)
    nb = _nrm(b)
    info = Info()
    if nb == 0.0:
        return np.zeros_like(b), info
    rnd = (lambda v: np.asarray(v, dtype=inner).astype(np.float64))
    A_in = A.astype(inner) if inner is not np.float64 else A
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - A @ x
    rn = _nrm(r)
    info.relres0 = info.relres = rn / nb
    info.history = []
    if rn <= rtol * nb:
        return x, info
    trigger = None if use_trigger else -1.0
    brk = 1e-7 if inner is np.float32 else 1e-14
    while True:
        if info.refinements >= max_refine:
            info.status = NOCONV
            break
        info.refinements += 1
        z = rnd(minv(rnd(r / rn)))
        beta = _nrm(z)
        if trigger is None:
            trigger = rtol * nb * beta
        V = np.zeros((m + 1, b.size))
        V[0] = rnd(z / beta)
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        converged = restarted = False
        for j in range(m):
            info.iters += 1
            Av = (A_in @ V[j].astype(inner)).astype(np.float64)
            w = rnd(minv(rnd(Av)))
            w0 = _nrm(w)
            h1 = V[: j + 1] @ w
            w = rnd(w - V[: j + 1].T @ h1)
            h2 = V[: j + 1] @ w
            w = rnd(w - V[: j + 1].T @ h2)
            col = np.zeros(m + 1)
            col[: j + 1] = h1 + h2
            hn = _nrm(w)
            col[j + 1] = hn
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
            est = rn * abs(g[j + 1])
            floor = hn <= brk * w0 or abs(g[j + 1]) <= rtol_inner * beta
            if floor or est <= trigger:
                y = _back_substitute(H[: j + 1, : j + 1], g[: j + 1])
                xc = x + rn * (V[: j + 1].T @ y)
                rc = b - A @ xc
                rcn = _nrm(rc)
                info.checks += 1
                if rcn <= rtol * nb:
                    x, rn, converged = xc, rcn, True
                    break
                if floor:
                    x, r, rn, restarted = xc, rc, rcn, True
                    break
                trigger = est * rtol * nb / rcn
            V[j + 1] = rnd(w / hn)
        if not converged and not restarted:
            y = _back_substitute(H[:m, :m], g[:m])
            x = x + rn * (V[:m].T @ y)
            r = b - A @ x
            rn = _nrm(r)
            converged = rn <= rtol * nb
        info.relres = rn / nb
        info.history.append(info.relres)
        if converged:
            break
    return x, info


def _back_substitute(R, g):
    k = g.size
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - R[i, i + 1:k] @ y[i + 1:k]) / R[i, i]
    return y
