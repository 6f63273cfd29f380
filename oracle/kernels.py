"""Kernel functions K(r) (matrix entries A_ij = K(|x_i - x_j|) for i != j).

* inv_r: 1/r, the 3D Laplace Green's function used on 2D points (Section 1,
  table of Green's functions).
* exp:   exp(-r / ell), the Ornstein-Uhlenbeck / exponential covariance
  (Section 1, table of covariance functions).
* dexp_dell: d/d ell of exp(-r / ell) = (r / ell^2) exp(-r / ell), the
  entries of dA/d ell for gradients with respect to the length scale.
* The three singular kernels of the numerical section, each continuous at
  r = a with K(a) = 1 (parameter a, passed as ``ell``):
  - log_a   (i):   r (log r - 1) / (a (log a - 1)) for r < a, log r / log a else;
  - inv_r_a (ii):  r / a for r < a, a / r else;
  - r2log_a (iii): r^3 (3 log r - 1) / (a^3 (3 log a - 1)) for r < a,
                   r^2 log r / (a^2 log a) else;
  their limits at r = 0 are 0 (two equal points).

A kernel is also allowed to be any callable taking two (n, 2) arrays of
points and returning the (n_a, n_b) matrix, which the tests use for
polynomial kernels that Chebyshev interpolation reproduces exactly.
"""
from __future__ import annotations

import numpy as np

KINDS = ("inv_r", "exp", "callable", "dexp_dell", "log_a", "inv_r_a", "r2log_a")


def radial(kind: str, a: float, r: np.ndarray) -> np.ndarray:
    """K(r) of a built-in kernel, elementwise."""
    r = np.asarray(r, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        if kind == "inv_r":
            return 1.0 / r
        if kind == "exp":
            return np.exp(-r / a)
        if kind == "dexp_dell":
            return r / (a * a) * np.exp(-r / a)
        small = r < a
        if kind == "log_a":
            near = r * (np.log(r) - 1.0) / (a * (np.log(a) - 1.0))
            far = np.log(r) / np.log(a)
        elif kind == "inv_r_a":
            near = r / a
            far = a / r
        elif kind == "r2log_a":
            near = r ** 3 * (3.0 * np.log(r) - 1.0) / (a ** 3 * (3.0 * np.log(a) - 1.0))
            far = r * r * np.log(r) / (a * a * np.log(a))
        else:
            raise ValueError(kind)
        out = np.where(small, near, far)
    return np.where(r == 0.0, 0.0, out)


class Kernel:
    def __init__(self, kind: str, ell: float = 0.0, fn=None):
        self.kind = kind
        self.ell = float(ell)
        self.fn = fn
        if kind not in KINDS:
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
        if self.kind == "exp":
            return np.exp(-r / self.ell)
        return radial(self.kind, self.ell, r)
