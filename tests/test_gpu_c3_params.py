"""GPU against the oracle at the 1M benchmark's parameters on a problem the
oracle factors in test time, element by element; and the caller-supplied
diagonal.

Benchmark parameters: exp(-r/0.1), A_ii = 1 + 1e-2, leaf 64, 6 x 6 Chebyshev
(rank 36), eps = 1e-8; here on 16,384 uniform points (4 levels).  Bars:
* FP64 factor, direct solve: ranks within +-1 of the oracle's on every
  cluster (different ones on < 2% of the clusters of each level); x within
  100 eps of the oracle's x (relative 2-norm) and 200 eps element by element
  (largest |x_i - xo_i| over the largest |xo_i|): two correct runs of the
  algorithm differ by rounding in the truncated directions, O(eps);
* refined to 1e-12 (FP64 factor) or 1e-10 (mixed-precision factor), x agrees
  with the oracle's refined solution element by element to 1e-7: the
  residual bound times the condition number (~2e4 here);
* the FMM product equals the oracle's to 1e-12.
Caller-supplied diagonal (IFMM_DIAG_VECTOR): the factor of A with A_ii = d_i
(a seeded vector) matches the oracle given the same vector, its diagonal and
FMM product are the vector and the oracle's product, and a constant vector
reproduces the constant-diagonal factor bit for bit.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle.ifmm import IFMM
from oracle.kernels import Kernel

pytestmark = pytest.mark.gpu

N16 = 16384
EPS = 1e-8


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _elem(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def oracle16k():
    _say(f"[gpu] oracle at the benchmark parameters, n={N16} (CPU, ~40 s)")
    pts = workloads.points_for("c3_exp_1m", N16)
    b = workloads.rhs_for("c3_exp_1m", N16)[:, 0].copy()
    o = IFMM(pts, Kernel("exp", 0.1), EPS, 64, 6, "const", 1.01).factor()
    assert o.tree.kappa == 4
    xo = o.solve(b)
    xr, hist = o.solve_refined(b, 1e-12)
    _say(f"  oracle: direct residual {hist[0]:.2e}, refined {hist[-1]:.2e} in {len(hist) - 1} sweeps")
    return pts, b, o, xo, xr


def _solver(torch_dev, pts, **kw):
    torch, dev = torch_dev
    from paper_1407_1572_amd import IFMMSolver
    return IFMMSolver(torch.from_numpy(pts).to(dev), "exp", 0.1, "const", 1.01, EPS, 64, 36, **kw)


def test_benchmark_parameters_fp64_elementwise(torch_dev, oracle16k):
    torch, dev = torch_dev
    pts, b, o, xo, xr = oracle16k
    _say("[gpu] benchmark parameters n=16384, FP64 factor, direct and refined")
    tb = torch.from_numpy(b).to(dev)
    s = _solver(torch_dev, pts)
    x = s.solve(tb).cpu().numpy()
    for k in range(2, o.tree.kappa + 1):
        d = np.abs(s.ranks(k) - o.r[k])
        _say(f"  level {k}: ranks differ on {(d > 0).sum()} of {len(d)} clusters (max {d.max()})")
        assert d.max() <= 1 and (d > 0).mean() < 0.02
    _say(f"  direct x vs oracle: 2-norm {_rel(x, xo):.2e}, element-wise {_elem(x, xo):.2e}")
    assert _rel(x, xo) < 100 * EPS and _elem(x, xo) < 200 * EPS
    y = s.matvec(tb).cpu().numpy()
    yo = o.apply(b)
    assert _rel(y, yo) < 1e-12 and _elem(y, yo) < 1e-12
    s.close()
    s = _solver(torch_dev, pts, refine_tol=1e-12)
    x = s.solve(tb).cpu().numpy()
    _say(f"  refined ({s.last_info['iterations']} sweeps, {s.last_info['residual']:.2e}): "
         f"x vs oracle's refined x: 2-norm {_rel(x, xr):.2e}, element-wise {_elem(x, xr):.2e}")
    assert s.last_info["residual"] <= 1e-12
    assert _elem(x, xr) < 1e-7
    s.close()


def test_benchmark_parameters_mixed_elementwise(torch_dev, oracle16k):
    torch, dev = torch_dev
    pts, b, o, xo, xr = oracle16k
    _say("[gpu] benchmark parameters n=16384, mixed-precision factor refined to 1e-10")
    s = _solver(torch_dev, pts, refine_tol=1e-10, precision="fp32")
    x = s.solve(torch.from_numpy(b).to(dev)).cpu().numpy()
    info = s.last_info
    res = np.linalg.norm(b - o.apply(x)) / np.linalg.norm(b)
    _say(f"  {info['iterations']} sweeps (direct {info['history'][0]:.2e}) to {info['residual']:.2e}; "
         f"oracle residual {res:.2e}; x vs oracle's refined x: 2-norm {_rel(x, xr):.2e}, "
         f"element-wise {_elem(x, xr):.2e}")
    assert info["residual"] <= 1e-10 and res <= 2e-10
    assert _elem(x, xr) < 1e-5 and _rel(x, xr) < 1e-5
    s.close()


def test_diagonal_vector(torch_dev):
    torch, dev = torch_dev
    _say("[gpu] caller-supplied diagonal, n=4096")
    n = 4096
    pts = workloads.uniform(n, 1013)
    d = 1.01 + 0.5 * np.random.default_rng(1014).uniform(size=n)
    b = workloads.rhs(n, 1, 2013)[:, 0].copy()
    tp, tb = torch.from_numpy(pts).to(dev), torch.from_numpy(b).to(dev)
    from paper_1407_1572_amd import IFMMSolver
    s = IFMMSolver(tp, "exp", 0.1, "vector", 0.0, EPS, 64, 36, diag_values=torch.from_numpy(d).to(dev))
    x = s.solve(tb).cpu().numpy()
    o = IFMM(pts, Kernel("exp", 0.1), EPS, 64, 6, "vector", 0.0, diag_values=d).factor()
    xo = o.solve(b)
    assert np.array_equal(s.diagonal().cpu().numpy(), d)
    y = s.matvec(tb).cpu().numpy()
    assert _elem(y, o.apply(b)) < 1e-12
    for k in range(2, o.tree.kappa + 1):
        dd = np.abs(s.ranks(k) - o.r[k])
        assert dd.max() <= 1 and (dd > 0).mean() < 0.02
    _say(f"  x vs oracle: 2-norm {_rel(x, xo):.2e}, element-wise {_elem(x, xo):.2e}")
    assert _rel(x, xo) < 100 * EPS and _elem(x, xo) < 200 * EPS
    s.close()
    # a constant vector is the constant diagonal, bit for bit
    s1 = IFMMSolver(tp, "exp", 0.1, "vector", 0.0, EPS, 64, 36,
                    diag_values=torch.full((n,), 1.01, dtype=torch.float64, device=dev))
    s2 = IFMMSolver(tp, "exp", 0.1, "const", 1.01, EPS, 64, 36)
    assert torch.equal(s1.solve(tb), s2.solve(tb))
    s1.close()
    s2.close()
    # a non-finite entry is refused
    from paper_1407_1572_amd import IFMMError
    bad = torch.from_numpy(d).to(dev)
    bad[77] = float("nan")
    with pytest.raises(IFMMError) as e:
        IFMMSolver(tp, "exp", 0.1, "vector", 0.0, EPS, 64, 36, diag_values=bad)
    assert e.value.code == 1


def test_rank_cap_hits_are_reported(torch_dev):
    """A cap that binds shows in the per-level cap-hit counts; an ample one
    does not."""
    torch, dev = torch_dev
    _say("[gpu] rank-cap hits: cap 16 (binds) against 128")
    pts = workloads.uniform(4096, 1003)
    tp = torch.from_numpy(pts).to(dev)
    from paper_1407_1572_amd import IFMMSolver
    s = IFMMSolver(tp, "exp", 0.1, "const", 1.01, EPS, 16, 16, r_max=16)
    hits = s.stats()["level_cap_hits"]
    s.close()
    s = IFMMSolver(tp, "exp", 0.1, "const", 1.01, 1e-4, 16, 16, r_max=128)
    none = s.stats()["level_cap_hits"]
    s.close()
    _say(f"  cap 16: {hits}; cap 128 at eps 1e-4: {none}")
    assert sum(hits.values()) > 0 and sum(none.values()) == 0
