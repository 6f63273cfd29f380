"""GPU: an exactly singular pivot block is reported as IFMM_ESINGULAR through
the C-ABI.  With a zero diagonal (IFMM_DIAG_VECTOR) and exp(-r/ell) at
ell = 1e-9, every off-diagonal entry of the FMM matrix underflows to 0, so
each leaf's pivot block [[P_ii, U], [U^T, 0]] is [[0, U], [U^T, 0]], of rank
at most 2 r < n + r: Gauss-Jordan meets an exact zero pivot once the r rows
of U^T are used.  The handle is not created, and the library still factors a
regular problem right after."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
IFMM_ESINGULAR = 3


def test_singular_pivot_block_is_reported():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1407_1572_amd.ifmm import _Kernel, load
    lib = load()
    dev = torch.device("cuda:0")
    n = 2048
    pts = torch.from_numpy(workloads.uniform(n, 9100)).to(dev)
    d = torch.zeros(n, dtype=torch.float64, device=dev)
    k = _Kernel(1, 1e-9, 2, 0.0, ctypes.c_void_p(d.data_ptr()))
    h = ctypes.c_void_p()
    torch.cuda.synchronize()
    print(f"[gpu] singular: N={n} exp ell=1e-9 zero diagonal, leaf 64, rank 16", flush=True)
    rc = lib.ifmm_factor(ctypes.c_void_p(pts.data_ptr()), n, ctypes.byref(k), 1e-6, 64, 16, None, None,
                         ctypes.byref(h))
    assert rc == IFMM_ESINGULAR, rc
    assert not h.value
    # a regular problem on the same points right after
    from paper_1407_1572_amd import IFMMSolver
    s = IFMMSolver(pts, "exp", 0.1, "const", 1.01, 1e-8, 64, 16, refine_tol=1e-10)
    b = torch.from_numpy(workloads.rhs(n, 1, 9101)[:, 0].copy()).to(dev)
    s.solve(b)
    assert s.last_info["status"] == 0 and s.last_info["residual"] <= 1e-10
    s.close()
