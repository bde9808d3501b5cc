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
* V = Q uses Householder QR without pivoting (numpy.linalg.qr); the least squares is the same
  column-scaled Householder QR with in-order drop as the EWMA path (``subspace.guess``).

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

    def __init__(self, n: int, K: int, k: int, seed: int, orthonormalize: bool = False):
        if not 1 <= k <= K:
            raise ValueError("need 1 <= k <= K")
        self.n, self.K, self.k, self.seed = n, K, k, seed
        self.orthonormalize = orthonormalize
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

    def basis(self) -> np.ndarray:
        """V = X Omega (n x k), or its orthonormal QR factor Q."""
        V = self.X() @ self.Omega()
        if self.orthonormalize:
            V, _ = np.linalg.qr(V)
        return V
