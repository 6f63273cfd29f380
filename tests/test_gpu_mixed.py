"""GPU: the mixed-precision factor (FP32 blocks, FP64 pivots / FMM / vectors)
refined in FP64 against the FMM matrix, compared with the FP64 path and the
dense FP64 solve.

Bars: the refined residual ||b - A x|| / ||b|| is recomputed on the CPU with
the oracle's FMM product and must meet the requested 1e-10; the error against
the dense FP64 solve is then bounded by cond(A) * 1e-10, checked at 1e-7
(these matrices have cond(A) < 1e3); the FP32 factor must also be a usable
preconditioner on its own (direct-solve residual < 1e-2, so refinement
contracts).
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import fmm_matrix as fm
from oracle.ifmm import IFMM
from oracle.kernels import Kernel

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


CASES = [
    # name, points, kernel, ell, diag, c0, eps, leaf, p
    ("c1_invr_2048_eps1e-6", lambda: workloads.points_for("c1_invr_2k"), "inv_r", 0.0, "rowsum", 1.0,
     1e-6, 32, 4),
    ("exp_4096_p6_eps1e-8", lambda: workloads.uniform(4096, 1003), "exp", 0.1, "const", 1.01, 1e-8, 64, 6),
    ("invr_4096_p6_eps1e-8", lambda: workloads.jittered_grid(4096, 1002), "inv_r", 0.0, "rowsum", 1.0,
     1e-8, 16, 6),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_mixed_refines_to_fp64_accuracy(torch_dev, case):
    name, mk, kind, ell, diag, c0, eps, leaf, p = case
    _say(f"[gpu] mixed precision {name}")
    torch, dev = torch_dev
    from paper_1407_1572_amd import IFMMSolver
    pts = mk()
    n = len(pts)
    B = workloads.rhs(n, 2, 2001)
    o = IFMM(pts, Kernel(kind, ell), eps, leaf, p, diag, c0)
    o.assemble()
    A = fm.dense_matrix(o.tree, o.kernel, p, diag, c0)
    xt = np.linalg.solve(A, B[o.tree.perm])
    xd = np.empty_like(xt)
    xd[o.tree.perm] = xt
    tp = torch.from_numpy(pts).to(dev)
    tb = torch.from_numpy(B).to(dev)
    s32 = IFMMSolver(tp, kind, ell, diag, c0, eps, leaf, p * p, precision="fp32")
    assert s32.stats()["precision"] == "fp32"
    x0 = s32.solve(tb).cpu().numpy()
    res0 = max(np.linalg.norm(B[:, j] - o.apply(x0[:, j])) / np.linalg.norm(B[:, j]) for j in range(2))
    assert res0 < 1e-2, res0
    s32.close()
    s32 = IFMMSolver(tp, kind, ell, diag, c0, eps, leaf, p * p, precision="fp32", refine_tol=1e-10)
    x = s32.solve(tb).cpu().numpy()
    info = s32.last_info
    res = max(np.linalg.norm(B[:, j] - o.apply(x[:, j])) / np.linalg.norm(B[:, j]) for j in range(2))
    err = np.linalg.norm(x - xd) / np.linalg.norm(xd)
    s64 = IFMMSolver(tp, kind, ell, diag, c0, eps, leaf, p * p, refine_tol=1e-10)
    x64 = s64.solve(tb).cpu().numpy()
    err64 = np.linalg.norm(x64 - xd) / np.linalg.norm(xd)
    _say(f"  direct residual {res0:.2e}; refined: {info['iterations']} sweeps, residual {res:.2e}, "
         f"error vs dense FP64 {err:.2e} (FP64 factor: {s64.last_info['iterations']} sweeps, {err64:.2e})")
    assert info["residual"] <= 1e-10 and res <= 2e-10
    assert err < 1e-7
    s32.close()
    s64.close()
