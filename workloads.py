"""Seeded synthetic inputs for the IFMM solver and its CPU oracle.

This module only draws random numbers; it holds none of the method's
arithmetic.  Both the oracle tests and the GPU tests / benchmark call it, so
the two sides always see bit-identical inputs.

Workloads (all points live in the unit square [0,1]^2):

* ``jittered_grid(n, seed)``  -- n_side = ceil(sqrt(n)), spacing h = 1/n_side,
  point i sits at ((i mod n_side) + 1/2, (i div n_side) + 1/2) * h plus a
  uniform offset in [-h/4, h/4]^2; the last grid row may be partial.  For
  n = 65536 this is the 256 x 256 jittered grid (exactly 64 points per leaf
  box at leaf size 64).
* ``uniform(n, seed)`` -- i.i.d. uniform points.  The paper's benchmark draws
  random points in a square such that the tree is balanced (Section 5); i.i.d.
  uniform points at the depth chosen from the mean leaf occupancy give that.
* ``rhs(n, nrhs, seed)`` -- standard normal right-hand sides, column-major
  [nrhs][n] as the C-ABI expects (returned as an (n, nrhs) Fortran array).

Seeds: points use 1000 + c and right-hand sides 2000 + c for the workload
numbered c (1-based) in the table below.
"""
from __future__ import annotations

import math

import numpy as np

# name -> (n, layout, kernel kind, ell, diag mode, c0, leaf, p, eps, nrhs)
# kernel kind: "inv_r" (1/r) or "exp" (exp(-r/ell)); diag mode "rowsum"
# (A_ii = c0 + sum_{j!=i} A_ij over the FMM matrix) or "const" (A_ii = c0).
WORKLOADS = {
    "c1_invr_2k": dict(cid=1, n=2048, layout="grid", kernel="inv_r", ell=0.0,
                       diag="rowsum", c0=1.0, leaf=32, p=4, eps=1e-6, nrhs=1),
    "c2_invr_64k": dict(cid=2, n=65536, layout="grid", kernel="inv_r", ell=0.0,
                        diag="rowsum", c0=1.0, leaf=64, p=6, eps=1e-8, nrhs=4),
    "c3_exp_1m": dict(cid=3, n=1 << 20, layout="uniform", kernel="exp", ell=0.1,
                      diag="const", c0=1.0 + 1e-2, leaf=64, p=6, eps=1e-8, nrhs=1),
}


def jittered_grid(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    side = int(math.ceil(math.sqrt(n)))
    h = 1.0 / side
    i = np.arange(n)
    base = np.stack([(i % side) + 0.5, (i // side) + 0.5], axis=1) * h
    jit = rng.uniform(-0.25 * h, 0.25 * h, size=(n, 2))
    return np.ascontiguousarray(base + jit, dtype=np.float64)


def uniform(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(0.0, 1.0, size=(n, 2)), dtype=np.float64)


def rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n, nrhs)))


def points_for(name: str, n: int | None = None) -> np.ndarray:
    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    gen = jittered_grid if w["layout"] == "grid" else uniform
    return gen(n, 1000 + w["cid"])


def rhs_for(name: str, n: int | None = None, nrhs: int | None = None) -> np.ndarray:
    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    nrhs = w["nrhs"] if nrhs is None else nrhs
    return rhs(n, nrhs, 2000 + w["cid"])
