"""Kernel functions K(r) (matrix entries A_ij = K(|x_i - x_j|) for i != j).

* inv_r: 1/r, the 3D Laplace Green's function used on 2D points (Section 1,
  table of Green's functions).
* exp:   exp(-r / ell), the Ornstein-Uhlenbeck / exponential covariance
  (Section 1, table of covariance functions).

A kernel is also allowed to be any callable taking two (n, 2) arrays of
points and returning the (n_a, n_b) matrix, which the tests use for
polynomial kernels that Chebyshev interpolation reproduces exactly.
"""
from __future__ import annotations

import numpy as np


class Kernel:
    def __init__(self, kind: str, ell: float = 0.0, fn=None):
        self.kind = kind
        self.ell = float(ell)
        self.fn = fn
        if kind not in ("inv_r", "exp", "callable"):
            raise ValueError(kind)

    def __call__(self, xa: np.ndarray, xb: np.ndarray) -> np.ndarray:
        xa = np.asarray(xa, dtype=np.float64).reshape(-1, 2)
        xb = np.asarray(xb, dtype=np.float64).reshape(-1, 2)
        if self.kind == "callable":
            return np.asarray(self.fn(xa, xb), dtype=np.float64)
        dx = xa[:, None, 0] - xb[None, :, 0]
        dy = xa[:, None, 1] - xb[None, :, 1]
        r = np.sqrt(dx * dx + dy * dy)
        if self.kind == "inv_r":
            with np.errstate(divide="ignore"):
                return 1.0 / r
        return np.exp(-r / self.ell)
