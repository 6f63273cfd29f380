"""GPU: ifmm_matvec_noalloc (the product with the library's fixed device
workspace, for callers that cannot allocate) against ifmm_matvec, through
the C-ABI: two calls in a row on one handle, the second with a smaller
input (fewer columns, then a second, smaller problem), each equal to
ifmm_matvec's result bit for bit (same kernels, same order of operations);
sizes beyond the workspace are refused.
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_matvec_noalloc_matches_matvec():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1407_1572_amd import IFMMError, IFMMSolver
    dev = torch.device("cuda:0")
    _say("[gpu] matvec without allocation: 65,536 points, 2 columns then 1; then 4,096 points")
    pts = workloads.points_for("c2_invr_64k")
    n = len(pts)
    s = IFMMSolver(torch.from_numpy(pts).to(dev), "inv_r", 0.0, "rowsum", 1.0, 1e-8, 64, 36)
    X = torch.from_numpy(np.ascontiguousarray(workloads.rhs(n, 2, 2301).T)).to(dev)  # [2][n]
    ref = s.matvec(X.t())  # [n, 2]
    out = torch.full((2, n), np.nan, dtype=torch.float64, device=dev)
    s.matvec_noalloc(X.t(), out.t())
    torch.cuda.synchronize()
    assert torch.equal(out.t(), ref)
    # second call, smaller input: one column
    x1 = X[1].clone()
    ref1 = s.matvec(x1)
    out1 = torch.full((n,), np.nan, dtype=torch.float64, device=dev)
    s.matvec_noalloc(x1, out1)
    torch.cuda.synchronize()
    assert torch.equal(out1, ref1)
    assert torch.equal(out1, ref[:, 1])
    # beyond the fixed workspace: refused, output untouched
    big = s.matvec_noalloc_bytes(64)
    assert big > 64 << 20
    x64 = torch.zeros((n, 64), dtype=torch.float64, device=dev)
    o64 = torch.full((64, n), 7.0, dtype=torch.float64, device=dev)
    with pytest.raises(IFMMError) as e:
        s.matvec_noalloc(x64, o64.t())
    assert e.value.code == 6
    assert bool((o64 == 7.0).all())
    s.close()
    # a smaller problem on another handle reuses the same workspace
    pts2 = workloads.uniform(4096, 1003)
    s2 = IFMMSolver(torch.from_numpy(pts2).to(dev), "exp", 0.1, "const", 1.01, 1e-8, 64, 36)
    x2 = torch.from_numpy(workloads.rhs(4096, 1, 2302)[:, 0].copy()).to(dev)
    out2 = torch.empty(4096, dtype=torch.float64, device=dev)
    s2.matvec_noalloc(x2, out2)
    torch.cuda.synchronize()
    assert torch.equal(out2, s2.matvec(x2))
    s2.close()
