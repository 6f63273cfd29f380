"""GPU: batched factor and solve of independent problems of uneven size
(ifmm_factor_batched / ifmm_solve_batched through the C-ABI).

Batch: 12 problems, N_j = round(exp(U(ln 1024, ln 32768))) (seed 4000 + j
points, uniform in [0,1]^2), kernels alternating between 1/r with the
row-sum diagonal (even j) and exp(-r/0.1) + 1e-2 I (odd j), leaf 64, 6 x 6
Chebyshev, eps 1e-8, 8 right-hand sides (seed 5000 + j), FP32 factor with
FP64 refinement to 1e-10, four host threads.  Bars:
* every batched factor, and every batched solve, equals the single-problem
  ifmm_factor / ifmm_solve of the same problem bit for bit (same kernels in
  the same order, only on another stream, concurrently with other problems);
* on the 8 smallest problems the refined solution matches the oracle's
  refined solution (FP64, 1e-12) element by element within 1e-6, and the
  oracle's FMM product gives a residual <= 2e-10.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle.ifmm import IFMM
from oracle.kernels import Kernel

pytestmark = pytest.mark.gpu
COUNT = 12


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _problems():
    out = []
    for j in range(COUNT):
        n = int(round(np.exp(np.random.default_rng(3000 + j).uniform(np.log(1024), np.log(32768)))))
        pts = workloads.uniform(n, 4000 + j)
        B = workloads.rhs(n, 8, 5000 + j)
        k = ({"kind": "inv_r", "ell": 0.0, "diag": "rowsum", "c0": 1.0} if j % 2 == 0 else
             {"kind": "exp", "ell": 0.1, "diag": "const", "c0": 1.01})
        out.append((pts, B, k))
    return out


def test_batched_equals_single_and_matches_oracle():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1407_1572_amd import IFMMSolver, factor_batched, solve_batched
    dev = torch.device("cuda:0")
    probs = _problems()
    _say(f"[gpu] batched: {COUNT} problems, N = {[len(p[0]) for p in probs]}")
    tp = [torch.from_numpy(p[0]).to(dev) for p in probs]
    tb = [torch.from_numpy(p[1]).to(dev) for p in probs]
    kw = dict(eps=1e-8, leaf_size=64, rank=36, refine_tol=1e-10, precision="fp32")
    sv = factor_batched(tp, [p[2] for p in probs], threads=4, **kw)
    X = solve_batched(sv, tb, threads=4)
    infos = [s.last_info for s in sv]
    assert all(i["status"] == 0 and i["residual"] <= 1e-10 for i in infos), infos
    for j, (pts, B, k) in enumerate(probs):
        s1 = IFMMSolver(tp[j], k["kind"], k["ell"], k["diag"], k["c0"], 1e-8, 64, 36, refine_tol=1e-10,
                        precision="fp32")
        for lvl in range(2, s1.stats()["kappa"] + 1):
            assert np.array_equal(s1.ranks(lvl), sv[j].ranks(lvl)), (j, lvl)
        x1 = s1.solve(tb[j])
        assert torch.equal(x1, X[j]), j
        s1.close()
    # the oracle on the 8 smallest problems
    small = sorted(range(COUNT), key=lambda j: len(probs[j][0]))[:8]
    for j in small:
        pts, B, k = probs[j]
        o = IFMM(pts, Kernel(k["kind"], k["ell"]), 1e-8, 64, 6, k["diag"], k["c0"]).factor()
        xo, hist = o.solve_refined(B, 1e-12)
        x = X[j].cpu().numpy()
        res = np.max(np.linalg.norm(B - o.apply(x), axis=0) / np.linalg.norm(B, axis=0))
        err = np.abs(x - xo).max() / np.abs(xo).max()
        _say(f"  problem {j} (N={len(pts)}, {k['kind']}): oracle residual {res:.2e}, element-wise vs oracle {err:.2e}")
        assert res <= 2e-10 and err <= 1e-6
    for s in sv:
        s.close()


def test_handles_outlive_the_streams_they_ran_on():
    """A factor built on a stream the caller then destroys is solved, used
    and destroyed on other streams (the library keeps no event of that
    stream alive across calls); batched calls back to back reuse their
    worker streams.  Regression: events recorded on a destroyed stream made
    later calls fail with a HIP error."""
    import ctypes

    import torch
    from paper_1407_1572_amd import IFMMSolver, factor_batched, solve_batched
    from paper_1407_1572_amd.ifmm import _Kernel, _Options, _SolveInfo, load
    _say("[gpu] handles outliving their streams")
    dev = torch.device("cuda:0")
    hip = ctypes.CDLL("libamdhip64.so")
    lib = load()
    pts = torch.from_numpy(workloads.uniform(4096, 1017)).to(dev)
    b = torch.from_numpy(workloads.rhs(4096, 1, 2017)[:, 0].copy()).to(dev)
    ref = IFMMSolver(pts, "exp", 0.1, "const", 1.01, 1e-8, 64, 36, refine_tol=1e-10)
    xr = ref.solve(b)
    torch.cuda.synchronize()
    for rep in range(3):
        st = ctypes.c_void_p()
        assert hip.hipStreamCreate(ctypes.byref(st)) == 0
        k = _Kernel(1, 0.1, 1, 1.01, ctypes.c_void_p(0))
        o = _Options()
        o.refine_tol = 1e-10
        h = ctypes.c_void_p()
        assert lib.ifmm_factor(ctypes.c_void_p(pts.data_ptr()), 4096, ctypes.byref(k), 1e-8, 64, 36, ctypes.byref(o),
                               st, ctypes.byref(h)) == 0
        x = torch.empty_like(b)
        info = _SolveInfo()
        assert lib.ifmm_solve(h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), 1, st,
                              ctypes.byref(info)) == 0
        assert hip.hipStreamDestroy(st) == 0
        x2 = torch.empty_like(b)
        assert lib.ifmm_solve(h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x2.data_ptr()), 1, None,
                              ctypes.byref(info)) == 0
        torch.cuda.synchronize()
        assert torch.equal(x, xr) and torch.equal(x2, xr)
        lib.ifmm_destroy(h)
    ref.close()
    # batched calls back to back
    probs = _problems()[:6]
    tp = [torch.from_numpy(p[0]).to(dev) for p in probs]
    tb = [torch.from_numpy(p[1][:, :2].copy()).to(dev) for p in probs]
    kw = dict(eps=1e-8, leaf_size=64, rank=36, refine_tol=1e-10, precision="fp32")
    first = None
    for rep in range(3):
        sv = factor_batched(tp, [p[2] for p in probs], threads=3, **kw)
        X = solve_batched(sv, tb, threads=3)
        X2 = solve_batched(sv, tb, threads=2)
        for a, c in zip(X, X2):
            assert torch.equal(a, c)
        if first is None:
            first = [x.clone() for x in X]
        for a, c in zip(X, first):
            assert torch.equal(a, c)
        for s in sv:
            s.close()
