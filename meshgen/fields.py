"""Seeded scalar fields used to build geometries and states.

``FourierField`` is the multi-scale random field of eq. (randfield) in
Sec. 4.3: a 2D Fourier sum with coefficients drawn uniformly from [-1, 1],
damped by |(j,k)|^-gamma (the pointwise uniform term is added by the caller,
per node).  ``vialov_dome`` is the dome thickness profile
H(r) = H0 (1 - r^{4/3})^{3/8}.
"""
from __future__ import annotations

import numpy as np


class FourierField:
    """s(x, y) = sum_{0<=j,k<=N, (j,k)!=(0,0)} (a,b,c,d).(cc, cs, sc, ss) |(j,k)|^-gamma, omega = 2 pi / L."""

    def __init__(self, rng: np.random.Generator, N: int, L: float, gamma: float = 1.5):
        self.N, self.L, self.gamma = N, L, gamma
        j = np.arange(N + 1, dtype=np.float64)
        jj, kk = np.meshgrid(j, j, indexing="ij")
        with np.errstate(divide="ignore"):
            damp = np.hypot(jj, kk) ** (-gamma)
        damp[0, 0] = 0.0
        coef = rng.uniform(-1.0, 1.0, size=(4, N + 1, N + 1))
        self.M = coef * damp[None]          # (a, b, c, d) damped, [4, N+1, N+1]

    def _tables(self, v: np.ndarray):
        w = 2.0 * np.pi / self.L
        arg = w * np.outer(v, np.arange(self.N + 1))
        return np.cos(arg), np.sin(arg)

    def grid(self, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
        """Field on the tensor grid xs x ys, [len(xs), len(ys)]."""
        Cx, Sx = self._tables(np.asarray(xs, dtype=np.float64))
        Cy, Sy = self._tables(np.asarray(ys, dtype=np.float64))
        A, B, C, D = self.M
        return Cx @ A @ Cy.T + Cx @ B @ Sy.T + Sx @ C @ Cy.T + Sx @ D @ Sy.T

    def __call__(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        """Field at scattered points, evaluated through the grid of their distinct x and y values."""
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        xs, ix = np.unique(x, return_inverse=True)
        ys, iy = np.unique(y, return_inverse=True)
        return self.grid(xs, ys)[ix.ravel(), iy.ravel()].reshape(x.shape)


def vialov_dome(r: np.ndarray, H0: float) -> np.ndarray:
    r = np.clip(np.asarray(r, dtype=np.float64), 0.0, 1.0)
    return H0 * np.clip(1.0 - r ** (4.0 / 3.0), 0.0, None) ** (3.0 / 8.0)
