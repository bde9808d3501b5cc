"""EWMA sketch and least-squares initial guess (test infrastructure, see package header).

Alg. 4 keeps a sketch Y = sum over stored solutions of r^(age) x omega^T (omega Gaussian in
R^k) and updates it after every solve by the rank-one recursion Y <- r^Delta Y + x omega^T
(Sec. 4.1.2). Alg. 2 takes V = Y (no orthonormalisation is needed, Sec. 4.1.1-4.1.2),
solves z* = argmin ||A V z - b|| by QR (Sec. 4) and starts GMRES from x0 = V z*.

Readings: Delta is one per stored solution (the forgetting exponent counts solves) by
default; with time labels (``push(x, tau)``, the option ``decay='time'``) it is the time since
the last stored solution in units of ``decay_dtau``, Alg. 4's exponent in physical time; the
least-squares problem is solved with Householder QR of the column-scaled W = A Y D
(D = diag(1/||W e_j||)) taken column by column in order, dropping a column whose norm
after projection out of the kept columns falls below ``tau_drop`` (the sketch becomes
ill-conditioned for small r, Sec. 5.1), so x0 = Y D z* over the kept columns.

Pins (tests/test_oracle_subspace.py): x0 equals the projection computed by numpy's
least-squares solver; an exact guess (zero GMRES steps) when the true solution lies in the
span of the history (the epsilon = 0 case of Thm. 4.1); Fischer's projection when A is
fixed and V = X (Sec. 4); the streaming recursion equals the explicit weighted sum; with
r = 0 the guess is the closed-form scaled last solution; span(Y) = span(Q) gives the same
guess for V = Y and V = Q.
"""
from __future__ import annotations

import numpy as np

from . import rng

TAU_DROP = 1e-7


class EWMASketch:
    """Y in R^{n x k}, zero until the first solution is pushed."""

    def __init__(self, n: int, k: int, r: float, seed: int, decay_dtau: float | None = None):
        self.Y = np.zeros((n, k))
        self.k, self.r, self.seed = k, float(r), seed
        self.decay_dtau = decay_dtau  # None: Delta = 1 per stored solution
        self.pushes = 0
        self.tau = None  # time label of the last stored solution

    def push(self, x, tau: float | None = None):
        w = np.array(rng.omega(self.seed, self.pushes, self.k))
        if self.decay_dtau is None:
            f = self.r
        else:
            f = self.r if self.pushes == 0 else self.r ** ((tau - self.tau) / self.decay_dtau)
            self.tau = tau
        self.Y = f * self.Y + np.outer(np.asarray(x, dtype=np.float64), w)
        self.pushes += 1


def householder_lstsq_drop(W, b, tau_drop: float = TAU_DROP, stats: dict | None = None):
    """Least squares min ||W z - b|| by Householder QR, columns in order, dropping any column
    whose projected norm |R_jj| < tau_drop * (norm of that column). Returns (z, kept) with z
    defined on the kept columns only. ``stats['margin']`` (when given) receives the smallest
    |ln(|R_jj| / (tau_drop ||W e_j||))| over the drop decisions."""
    W = np.array(W, dtype=np.float64, copy=True)
    n, k = W.shape
    reflectors = []  # (v, beta) acting on rows rank..n-1
    kept, rdiag, rcols = [], [], []
    for j in range(k):
        col = W[:, j].copy()
        cn = np.sqrt(col @ col)
        if cn == 0.0:
            continue
        for (rank0, v, beta) in reflectors:
            col[rank0:] -= beta * v * (v @ col[rank0:])
        rank = len(kept)
        tail = col[rank:]
        tn = np.sqrt(tail @ tail)
        if stats is not None and tn > 0.0:
            stats["margin"] = min(stats.get("margin", np.inf), abs(float(np.log(tn / (tau_drop * cn)))))
        if tn < tau_drop * cn:
            continue
        alpha = -tn if tail[0] >= 0.0 else tn
        v = tail.copy()
        v[0] -= alpha
        beta = 2.0 / (v @ v)
        reflectors.append((rank, v, beta))
        rcol = np.zeros(k)
        rcol[:rank] = col[:rank]
        rcol[rank] = alpha
        rcols.append(rcol)
        kept.append(j)
    if not kept:
        return np.zeros(0), kept
    qtb = np.array(b, dtype=np.float64, copy=True)
    for (rank0, v, beta) in reflectors:
        qtb[rank0:] -= beta * v * (v @ qtb[rank0:])
    m = len(kept)
    R = np.array(rcols).T[:m, :m]
    z = np.zeros(m)
    for i in range(m - 1, -1, -1):
        z[i] = (qtb[i] - R[i, i + 1:] @ z[i + 1:]) / R[i, i]
    return z, kept


def guess(A, Y, b, tau_drop: float = TAU_DROP, stats: dict | None = None):
    """x0 = Y D z* with z* = argmin ||A Y D z - b|| (Alg. 2 with V = Y, column-scaled).
    ``stats`` receives the margin of the drop decisions (householder_lstsq_drop)."""
    W = A @ Y
    norms = np.sqrt(np.einsum("ij,ij->j", W, W))
    scale = np.where(norms > 0.0, 1.0 / np.where(norms > 0.0, norms, 1.0), 0.0)
    z, kept = householder_lstsq_drop(W * scale[None, :], b, tau_drop, stats)
    x0 = np.zeros(Y.shape[0])
    if kept:
        x0 = Y[:, kept] @ (z * scale[kept])
    return x0, len(kept)
