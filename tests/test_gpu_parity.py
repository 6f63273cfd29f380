"""GPU parity: the HIP IFMM through the C-ABI against the CPU oracle.

Every case is seeded and synthetic.  Bars:
* eps = 0 (lossless compression): x equals the dense LU solve of the FMM
  matrix to 1e-11 relative -- FP64 round-off through ~3 levels of
  eliminations;
* eps > 0: same ranks as the oracle cluster by cluster (+-1 tolerated where a
  pivot norm sits at the threshold) and x within 50 eps of the oracle's x
  (relative 2-norm) and within 100 eps element by element (largest
  |x_i - xo_i| over the largest |xo_i|, so an error confined to a few clusters
  cannot hide in the norm); residual against the FMM matrix <= 10 eps;
* the FMM product and the assembled diagonal agree with the oracle to 1e-12;
* refinement reaches 1e-12.
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


def _gpu(torch_dev, pts, kind, ell, diag, c0, eps, leaf, p, **kw):
    torch, dev = torch_dev
    from paper_1407_1572_amd import IFMMSolver
    return IFMMSolver(torch.from_numpy(pts).to(dev), kind, ell, diag, c0, eps, leaf, p * p, **kw)


def _dense(o, b):
    A = fm.dense_matrix(o.tree, o.kernel, o.p, o.diag_mode, o.c0)
    xt = np.linalg.solve(A, b.reshape(o.tree.N, -1)[o.tree.perm])
    x = np.empty_like(xt)
    x[o.tree.perm] = xt
    return x.reshape(b.shape)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _elem(a, b):
    """Largest entry-wise difference relative to the largest entry."""
    return float(np.abs(a - b).max() / np.abs(b).max())


CASES_EXACT = [
    # name, points, kernel, ell, diag, c0, leaf, p, r_max
    ("invr_512_p3_3lev", lambda: workloads.jittered_grid(512, 1001), "inv_r", 0.0, "rowsum", 1.0, 8, 3, 64),
    ("exp_1500_p3_4lev", lambda: workloads.uniform(1500, 77), "exp", 0.1, "const", 1.01, 8, 3, 128),
]


@pytest.mark.parametrize("case", CASES_EXACT, ids=[c[0] for c in CASES_EXACT])
def test_eps0_matches_dense_solve(torch_dev, case):
    name, mk, kind, ell, diag, c0, leaf, p, rmax = case
    _say(f"[gpu] eps=0 exactness {name}")
    torch, dev = torch_dev
    pts = mk()
    b = workloads.rhs(len(pts), 2, 31)
    s = _gpu(torch_dev, pts, kind, ell, diag, c0, 0.0, leaf, p, r_max=rmax)
    x = s.solve(torch.from_numpy(b).to(dev)).cpu().numpy()
    o = IFMM(pts, Kernel(kind, ell), 0.0, leaf, p, diag, c0, r_cap=rmax)
    xd = _dense(o, b)
    assert _rel(x, xd) < 1e-11 and _elem(x, xd) < 1e-11
    o.factor()
    for k in range(2, o.tree.kappa + 1):
        assert np.array_equal(s.ranks(k), o.r[k]), k
    s.close()


CASES_EPS = [
    # name, points, kernel, ell, diag, c0, eps, leaf, p, residual bound of the
    # direct solve (10 eps unless the default rank cap 2p^2 binds)
    ("c1_invr_2048_eps1e-6", lambda: workloads.points_for("c1_invr_2k"), "inv_r", 0.0, "rowsum", 1.0,
     1e-6, 32, 4, 1e-5),
    ("exp_4096_eps1e-8_4lev_capped", lambda: workloads.uniform(4096, 1003), "exp", 0.1, "const", 1.01,
     1e-8, 16, 4, 1e-3),
    ("invr_4096_p6_eps1e-8", lambda: workloads.jittered_grid(4096, 1002), "inv_r", 0.0, "rowsum", 1.0,
     1e-8, 16, 6, 1e-7),
]


@pytest.mark.parametrize("case", CASES_EPS, ids=[c[0] for c in CASES_EPS])
def test_eps_matches_oracle(torch_dev, case):
    name, mk, kind, ell, diag, c0, eps, leaf, p, res_bound = case
    _say(f"[gpu] eps>0 parity {name}")
    torch, dev = torch_dev
    pts = mk()
    b = workloads.rhs(len(pts), 1, 2001)[:, 0]
    s = _gpu(torch_dev, pts, kind, ell, diag, c0, eps, leaf, p)
    x = s.solve(torch.from_numpy(b).to(dev)).cpu().numpy()
    o = IFMM(pts, Kernel(kind, ell), eps, leaf, p, diag, c0).factor()
    xo = o.solve(b)
    for k in range(2, o.tree.kappa + 1):
        d = np.abs(s.ranks(k) - o.r[k])
        assert d.max() <= 1 and (d > 0).mean() < 0.02, (k, d.max(), (d > 0).mean())
    _say(f"  x vs oracle: 2-norm {_rel(x, xo):.2e}, element-wise {_elem(x, xo):.2e}")
    assert _rel(x, xo) < 50 * eps and _elem(x, xo) < 100 * eps
    res = np.linalg.norm(b - o.apply(x)) / np.linalg.norm(b)
    assert res < res_bound
    # FMM product and diagonal
    y = s.matvec(torch.from_numpy(b).to(dev)).cpu().numpy()
    yo = o.apply(b)
    assert _rel(y, yo) < 1e-12 and _elem(y, yo) < 1e-12
    dg = s.diagonal().cpu().numpy()
    do = np.empty(len(pts))
    do[o.tree.perm] = o.d
    assert _rel(dg, do) < 1e-13
    s.close()


def test_multi_rhs_refinement_and_empty_leaves(torch_dev):
    _say("[gpu] refinement, 3 rhs, empty leaves")
    torch, dev = torch_dev
    rng = np.random.default_rng(5)
    n = 3000
    pts = np.column_stack([rng.uniform(0, 0.6, n), rng.uniform(0, 1, n)])
    B = rng.standard_normal((n, 3))
    s = _gpu(torch_dev, pts, "exp", 0.1, "const", 1.01, 1e-8, 16, 4, refine_tol=1e-12)
    X = s.solve(torch.from_numpy(B).to(dev)).cpu().numpy()
    info = s.last_info
    assert info["residual"] <= 1e-12 and info["iterations"] >= 1
    o = IFMM(pts, Kernel("exp", 0.1), 1e-8, 16, 4, "const", 1.01)
    xd = _dense(o, B)
    assert _rel(X, xd) < 1e-9 and _elem(X, xd) < 1e-9
    for j in range(3):  # column-wise agreement with single-rhs solves
        xj = s.solve(torch.from_numpy(B[:, j].copy()).to(dev)).cpu().numpy()
        assert _rel(xj, X[:, j]) < 1e-12
    s.close()


def test_profile_family_mask(torch_dev):
    _say("[gpu] profile: every family, then the elimination steps only")
    torch, dev = torch_dev
    from paper_1407_1572_amd import IFMMSolver
    pts = workloads.uniform(4096, 1003)
    tp = torch.from_numpy(pts).to(dev)
    b = torch.from_numpy(workloads.rhs(4096, 1, 2001)[:, 0].copy()).to(dev)
    counts = {}
    for prof in (True, ["elim"]):
        s = IFMMSolver(tp, "exp", 0.1, "const", 1.01, 1e-8, 64, 36, profile=prof)
        s.solve(b)
        k = {n: v for n, v in s.stats()["kernels"].items() if v["launches"] > 0}
        counts[str(prof)] = k
        s.close()
    full, only = counts["True"], counts["['elim']"]
    assert {"elim", "inverse", "rrqr", "solve"} <= set(full)
    assert set(only) == {"elim"}
    # the same launches, with the same algorithmic counts
    assert only["elim"]["launches"] == full["elim"]["launches"]
    assert only["elim"]["flops"] == full["elim"]["flops"] and only["elim"]["bytes"] == full["elim"]["bytes"]


def test_rejected_points(torch_dev):
    """Points the tree build refuses (not finite, outside the box, two equal
    points of the singular kernel) give 'invalid argument'; equal points are
    fine for the smooth kernel, and a point on the box's far edge is inside."""
    _say("[gpu] tree build: rejected points")
    from paper_1407_1572_amd import IFMMError
    base = workloads.uniform(600, 1007)
    bad = []
    p = base.copy(); p[17] = (1.25, 0.5); bad.append(("outside", p, "exp"))
    p = base.copy(); p[301, 1] = np.nan; bad.append(("nan", p, "exp"))
    p = base.copy(); p[5] = p[444]; bad.append(("equal, 1/r", p, "inv_r"))
    for name, pts, kern in bad:
        _say(f"  {name}")
        with pytest.raises(IFMMError) as e:
            _gpu(torch_dev, pts, kern, 0.1, "rowsum", 1.0, 1e-8, 8, 3, box=(0.0, 0.0, 1.0))
        assert e.value.code == 1
    p = base.copy(); p[5] = p[444]; p[9] = (1.0, 1.0)
    s = _gpu(torch_dev, p, "exp", 0.1, "const", 1.01, 0.0, 8, 3, r_max=64, box=(0.0, 0.0, 1.0))
    b = workloads.rhs(600, 1, 2003)[:, 0].copy()
    x = s.solve(torch_dev[0].from_numpy(b).to(torch_dev[1])).cpu().numpy()
    o = IFMM(p, Kernel("exp", 0.1), 0.0, 8, 3, "const", 1.01, r_cap=64)
    assert _rel(x, _dense(o, b)) < 1e-9
    s.close()


def test_nonfinite_rhs_is_not_converged(torch_dev):
    """A right-hand side with a NaN gives a NaN residual: refinement stops at
    once with 'did not converge' instead of reporting success."""
    _say("[gpu] refinement: NaN right-hand side")
    torch, dev = torch_dev
    pts = workloads.uniform(1024, 1009)
    s = _gpu(torch_dev, pts, "exp", 0.1, "const", 1.01, 1e-8, 16, 4, refine_tol=1e-10)
    b = workloads.rhs(1024, 1, 2005)[:, 0].copy()
    b[100] = np.nan
    s.solve(torch.from_numpy(b).to(dev), check=False)
    info = s.last_info
    assert info["status"] == 4 and info["iterations"] == 0 and not np.isfinite(info["residual"])
    b[100] = 0.5  # the same handle still solves a finite system
    s.solve(torch.from_numpy(b).to(dev))
    assert s.last_info["status"] == 0 and s.last_info["residual"] <= 1e-10
    s.close()


def test_five_rhs_and_plan_reuse(torch_dev):
    """Five right-hand sides (column groups of four and one in the solve
    kernels), then one column, then five again on the same handle: every
    solve matches the dense solve, and the single-column solve matches the
    corresponding column of the five-column one."""
    _say("[gpu] 5 rhs, then 1, then 5 on one handle")
    torch, dev = torch_dev
    pts = workloads.uniform(1500, 1011)
    B = workloads.rhs(1500, 5, 2007)
    # eps = 0 with a rank cap that never binds: lossless compression
    s = _gpu(torch_dev, pts, "exp", 0.1, "const", 1.01, 0.0, 8, 3, r_max=128)
    o = IFMM(pts, Kernel("exp", 0.1), 0.0, 8, 3, "const", 1.01, r_cap=128)
    xd = _dense(o, B)
    X = s.solve(torch.from_numpy(np.ascontiguousarray(B)).to(dev)).cpu().numpy()
    assert _rel(X, xd) < 1e-10 and _elem(X, xd) < 1e-10
    x2 = s.solve(torch.from_numpy(B[:, 2].copy()).to(dev)).cpu().numpy()
    assert _rel(x2, X[:, 2]) < 1e-12
    X2 = s.solve(torch.from_numpy(np.ascontiguousarray(B)).to(dev)).cpu().numpy()
    assert _rel(X2, X) < 1e-13
    s.close()
