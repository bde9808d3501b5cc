"""Randomized range finder over a sliding window of solutions (test infrastructure, see
package header).

Alg. 3 (Sec. 4.1.1) takes the K most recent solutions X = X(I) in R^{n x K}, draws a Gaussian
Omega in R^{K x k} (k <= K), forms the sketch V = X Omega and optionally replaces it by the
orthonormal factor Q of its QR decomposition; Alg. 2 then takes x0 from the least-squares
problem on A V. Readings:

* the window holds the K most recent stored solutions (every returned solution is stored, as
  for Alg. 4), oldest first;
* the row of Omega that belongs to a stored solution is drawn once, when the solution enters
  the window, from the same counter-based stream as Alg. 4's omega (``rng.omega`` of the
  solution's index), so V slides with the window as the paper's rank-1 updates of X Omega
  would;
* V = Q is the QR of the column-scaled sketch taken column by column in order (Gram-Schmidt
  applied twice), dropping a column whose norm after projection out of the kept ones falls
  below ``tau_drop`` (the least squares' own drop rule), so that Q spans the sketch's numerical
  range (a window with fewer solutions than k gives fewer columns, not directions of rounding
  noise); the least squares is the same column-scaled Householder QR with in-order drop as the
  EWMA path (``subspace.guess``).

Pins (tests/test_oracle_rangefinder.py): solutions that left the window have no component in
V; V has the rank min(k, window) of a full-rank window; x0 with V = Q equals x0 with V = X Omega
(same span) on a well-conditioned window; Fischer's projection for a fixed A when k = K
(Sec. 4: A x0 is the orthogonal projection of b onto span(A X)); an exact guess (zero GMRES
steps) when the true solution lies in the span of the window.
"""
from __future__ import annotations

from collections import deque

import numpy as np

from . import rng


class RangeFinder:
    """Sliding window of the K most recent solutions and their rows of Omega."""

    def __init__(self, n: int, K: int, k: int, seed: int, orthonormalize: bool = False,
                 tau_drop: float = 1e-7):
        if not 1 <= k <= K:
            raise ValueError("need 1 <= k <= K")
        self.n, self.K, self.k, self.seed = n, K, k, seed
        self.orthonormalize, self.tau_drop = orthonormalize, tau_drop
        self.window = deque()  # (solution, its row of Omega), oldest first
        self.pushes = 0

    def push(self, x):
        row = np.array(rng.omega(self.seed, self.pushes, self.k))
        self.window.append((np.array(x, dtype=np.float64, copy=True), row))
        if len(self.window) > self.K:
            self.window.popleft()
        self.pushes += 1

    def X(self) -> np.ndarray:
        return np.column_stack([x for x, _ in self.window])

    def Omega(self) -> np.ndarray:
        return np.vstack([row for _, row in self.window])

    def basis(self, stats: dict | None = None) -> np.ndarray:
        """V = X Omega (n x k), or its orthonormal QR factor Q (``stats['margin']`` then also
        receives the margins of its drop decisions)."""
        V = self.X() @ self.Omega()
        if self.orthonormalize:
            V = orthonormal_columns(V, self.tau_drop, stats)
        return V


def orthonormal_columns(V, tau_drop: float, stats: dict | None = None) -> np.ndarray:
    """Q with orthonormal columns: each column of V scaled to unit norm, projected out of the
    columns kept so far twice (classical Gram-Schmidt, second pass for the rounding of the
    first), kept when the norm left is at least tau_drop. ``stats['margin']`` (when given)
    receives the smallest |ln(norm left / tau_drop)| of the decisions."""
    qs = []
    for j in range(V.shape[1]):
        v = V[:, j]
        nv = np.linalg.norm(v)
        if nv == 0.0:
            continue
        w = v / nv
        for _ in range(2):
            if qs:
                Q = np.column_stack(qs)
                w = w - Q @ (Q.T @ w)
        nw = np.linalg.norm(w)
        if stats is not None and nw > 0.0:
            stats["margin"] = min(stats.get("margin", np.inf), abs(float(np.log(nw / tau_drop))))
        if nw >= tau_drop:
            qs.append(w / nw)
    return np.column_stack(qs) if qs else np.zeros((V.shape[0], 0))
