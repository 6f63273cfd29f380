"""GPU: the 65,536-point 1/r problem (256 x 256 jittered grid, A_ii = 1 +
FMM row sum, leaf 64, p = 6, eps = 1e-8, 4 right-hand sides) at full size,
FP64 factor and mixed-precision factor, both refined to 1e-10.

The oracle cannot factor this size in test time, so the checks use what it
can compute here: its FMM product and row-sum diagonal (the matrix both sides
solve with).  Bars:
* the diagonal assembled on the GPU equals the oracle's to 1e-12;
* the refined residual ||B - A X|| / ||B||, recomputed with the oracle's
  FMM product, meets 1e-10 for both factors (the refinement gate);
* the FP64 factor's direct solve (before refinement) has residual <= 10 eps
  per column, the compression accuracy gate;
* the mixed and FP64 solutions agree to 1e-8 (this matrix is diagonally
  dominant, cond(A) < 1e2, so a 1e-10 residual pins x to ~1e-8).
"""
import sys

import numpy as np
import pytest

import workloads
from oracle.fmm_matrix import diagonal, fmm_apply_offdiag
from oracle.geometry import Tree
from oracle.kernels import Kernel

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_c2_full_size_fp64_and_mixed():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1407_1572_amd import IFMMSolver
    dev = torch.device("cuda:0")
    w = workloads.WORKLOADS["c2_invr_64k"]
    pts = workloads.points_for("c2_invr_64k")
    B = workloads.rhs_for("c2_invr_64k")
    n = len(pts)
    _say(f"[gpu] C2 full size: n={n}, 4 rhs")
    tp = torch.from_numpy(pts).to(dev)
    tb = torch.from_numpy(B).to(dev)
    args = ("inv_r", 0.0, "rowsum", 1.0, w["eps"], w["leaf"], w["p"] ** 2)
    s64 = IFMMSolver(tp, *args, refine_tol=1e-10)
    X64 = s64.solve(tb).cpu().numpy()
    i64 = s64.last_info
    dg = s64.diagonal().cpu().numpy()
    s32 = IFMMSolver(tp, *args, refine_tol=1e-10, precision="fp32")
    X32 = s32.solve(tb).cpu().numpy()
    i32 = s32.last_info
    _say(f"  fp64: direct residual {i64['history'][0]:.2e}, {i64['iterations']} sweeps to {i64['residual']:.2e}")
    _say(f"  fp32: direct residual {i32['history'][0]:.2e}, {i32['iterations']} sweeps to {i32['residual']:.2e}")

    T = Tree(pts, w["leaf"])
    kern = Kernel("inv_r")
    d = diagonal(fmm_apply_offdiag(T, kern, w["p"], np.ones(n)), "rowsum", 1.0)
    do = np.empty(n)
    do[T.perm] = d
    assert np.abs(dg - do).max() / np.abs(do).max() < 1e-12

    def resid(X):
        Xt = X[T.perm]
        Y = fmm_apply_offdiag(T, kern, w["p"], Xt) + d[:, None] * Xt
        R = B[T.perm] - Y
        return np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)

    r64, r32 = resid(X64), resid(X32)
    diff = np.linalg.norm(X32 - X64) / np.linalg.norm(X64)
    _say(f"  oracle residual fp64 {r64.max():.2e}, fp32 {r32.max():.2e}; mixed vs fp64 {diff:.2e}")
    assert i64["history"][0] <= 10 * w["eps"]
    assert r64.max() <= 2e-10 and r32.max() <= 2e-10
    assert diff < 1e-8
    s64.close()
    s32.close()
