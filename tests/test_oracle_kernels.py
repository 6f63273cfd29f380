"""Pins for oracle/kernels.py: the numerical section's three singular
kernels and the exp kernel's length-scale derivative, from closed forms.

* each singular kernel is continuous at r = a with K(a) = 1, and tends to 0
  as r -> 0 (equal points);
* special values: log r / log a vanishes at r = 1; a / r is a at r = 1 and
  a / 2 at r = 2; r^2 log r / (a^2 log a) vanishes at r = 1 and equals
  4 log 2 / (a^2 log a) at r = 2; below a, r / a is linear;
* d/d ell exp(-r/ell) matches a central finite difference in ell;
* the lossless factorisation (eps = 0) of each kernel's FMM matrix with the
  numerical section's unit diagonal and root box [-1, 1]^2 equals the dense
  solve (the same pin as for the other kernels).
"""
import numpy as np
import pytest

import workloads
from oracle import fmm_matrix as fm
from oracle.ifmm import IFMM
from oracle.kernels import Kernel, radial

A = 1e-3


@pytest.mark.parametrize("kind", ["log_a", "inv_r_a", "r2log_a"])
def test_continuous_at_a_and_zero_at_the_origin(kind):
    below = radial(kind, A, np.array([A * (1 - 1e-9)]))[0]
    above = radial(kind, A, np.array([A * (1 + 1e-9)]))[0]
    assert abs(below - 1.0) < 1e-7 and abs(above - 1.0) < 1e-7
    assert radial(kind, A, np.array([0.0]))[0] == 0.0
    assert abs(radial(kind, A, np.array([1e-12]))[0]) < 1e-6


def test_special_values():
    assert radial("log_a", A, np.array([1.0]))[0] == 0.0
    assert np.isclose(radial("log_a", A, np.array([0.1]))[0], np.log(0.1) / np.log(A), rtol=1e-15)
    assert np.isclose(radial("inv_r_a", A, np.array([1.0, 2.0]))[0], A)
    assert np.isclose(radial("inv_r_a", A, np.array([2.0]))[0], A / 2)
    r = np.array([0.25e-3, 0.5e-3])
    assert np.allclose(radial("inv_r_a", A, r), r / A, rtol=1e-15)
    assert radial("r2log_a", A, np.array([1.0]))[0] == 0.0
    assert np.isclose(radial("r2log_a", A, np.array([2.0]))[0], 4 * np.log(2) / (A * A * np.log(A)), rtol=1e-14)


def test_length_scale_derivative():
    r = np.linspace(0.0, 0.5, 101)
    for ell in (0.08, 0.1):
        h = 1e-6 * ell
        fd = (np.exp(-r / (ell + h)) - np.exp(-r / (ell - h))) / (2 * h)
        assert np.allclose(radial("dexp_dell", ell, r), fd, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("kind", ["log_a", "inv_r_a", "r2log_a"])
def test_eps0_factor_of_the_numerical_section_kernels(kind):
    pts = 2.0 * workloads.uniform(1024, 91) - 1.0
    o = IFMM(pts, Kernel(kind, A), 0.0, 16, 4, "const", 1.0, r_cap=10 ** 6, lo=(-1.0, -1.0), size=2.0).factor()
    b = workloads.rhs(1024, 1, 92)[:, 0]
    Ad = fm.dense_matrix(o.tree, o.kernel, o.p, "const", 1.0)
    xt = np.linalg.solve(Ad, b[o.tree.perm])
    xd = np.empty_like(xt)
    xd[o.tree.perm] = xt
    x = o.solve(b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10 * max(1.0, np.linalg.cond(Ad)) ** 0.5


def test_fmm_matrix_derivative_is_the_fmm_matrix_of_the_kernel_derivative():
    # the Chebyshev FMM matrix is linear in the kernel, so d/d ell of the
    # matrix of exp(-r/ell) is the matrix of (r/ell^2) exp(-r/ell): checked
    # against a central difference of the dense matrices
    from oracle.geometry import Tree
    pts = workloads.uniform(600, 95)
    T = Tree(pts, 16)
    ell, h = 0.08, 1e-6
    dA = fm.dense_offdiag(T, Kernel("dexp_dell", ell), 4)
    fd = (fm.dense_offdiag(T, Kernel("exp", ell + h), 4) - fm.dense_offdiag(T, Kernel("exp", ell - h), 4)) / (2 * h)
    assert np.abs(dA - fd).max() <= 1e-7 * np.abs(dA).max()
    # and the FMM passes reproduce it
    x = workloads.rhs(600, 1, 96)[:, 0]
    assert np.allclose(fm.fmm_apply_offdiag(T, Kernel("dexp_dell", ell), 4, x), dA @ x, rtol=0,
                       atol=1e-12 * np.abs(dA @ x).max())
