"""Pins of the oracle's Theorem-3 pieces (CPU only).

* Second derivatives of the regularised delta/delta' weights satisfy the
  twice-differentiated moment conditions; wavelet second derivatives match
  differences of the first ones.
* H_1 + H_2 (Theorem 2) is the exact Hessian of the data misfit
  1/2 sum |y - g(theta)|^2 / sigma^2, so it must equal central differences
  of the misfit's gradient (computed from sensitivity solves) to O(d^2).
* Gauss-Newton stops where that gradient vanishes.
* On a linear-Gaussian model Theorem 3 is exact: averaged over theta* and y
  it equals 1/2 log det(I + Gamma H_1).
"""
import math

import numpy as np
import pytest

from oracle import elastic, laplace, theorem3
from synthetic import Grid, layered_medium

H = 9.0


@pytest.mark.parametrize("alpha", [0.0, 0.21, 0.5, 0.93])
def test_weight_second_derivatives_by_moments(alpha):
    # d^2/dx_s^2 of sum_j w_j (x_j - x_s)^p h = const gives
    # sum_j w''_j (x_j - x_s)^p h = p (p-1) sum_j w_j (x_j - x_s)^(p-2) h
    d_polys, dp_polys = elastic.weight_polys()
    rel = (np.arange(-2, 4) - alpha) * H
    for polys, scale in ((d_polys, 1 / H), (dp_polys, 1 / H**2)):
        w = np.array([p(alpha) for p in polys]) * scale
        w2 = np.array([p.deriv(2)(alpha) for p in polys]) * scale / H**2
        assert abs(H * np.sum(w2)) < 1e-9 * np.max(np.abs(w2)) * H
        assert abs(H * np.sum(w2 * rel)) < 1e-9 * np.max(np.abs(w2)) * H**2
        for p in range(2, 5):
            lhs = H * np.sum(w2 * rel**p)
            rhs = p * (p - 1) * H * np.sum(w * rel ** (p - 2))
            assert abs(lhs - rhs) < 1e-9 * max(1.0, abs(rhs)), (p, lhs, rhs)


def test_window_derivative_orders():
    th = np.array([317.3, 420.8, 0.1, 9.0, 1e13, -2e13, 5e13])
    for j in (0, 1):
        a = elastic.dsource_window(th, 16.0, j)[2]
        b = theorem3.window_derivative(th, 16.0, int(j == 0), int(j == 1))[2]
        assert np.allclose(a, b, rtol=1e-13, atol=0)
    # mixed second derivative by differences of the first
    e = 1e-3
    for (ox, oz, j) in ((2, 0, 0), (1, 1, 1), (0, 2, 1)):
        tp, tm = th.copy(), th.copy()
        tp[j] += e
        tm[j] -= e
        ax = int(ox - (j == 0))
        az = int(oz - (j == 1))
        num = (theorem3.window_derivative(tp, 16.0, ax, az)[2]
               - theorem3.window_derivative(tm, 16.0, ax, az)[2]) / (2 * e)
        ana = theorem3.window_derivative(th, 16.0, ox, oz)[2]
        assert np.max(np.abs(num - ana)) < 1e-5 * np.max(np.abs(ana))


@pytest.mark.parametrize("kind,p", [("gauss", 6.0), ("gauss_deriv", 7.5)])
def test_wavelet_second_derivatives(kind, p):
    t = np.linspace(0, 1.2, 601)
    t0, e = 0.4, 1e-5
    for wrt, (a, b) in (("t0t0", ("t0", "t0")), ("t0p", ("t0", "p")), ("pp", ("p", "p"))):
        if b == "t0":
            num = (elastic.dstf(t, t0 + e, p, kind, a) - elastic.dstf(t, t0 - e, p, kind, a)) / (2 * e)
        else:
            num = (elastic.dstf(t, t0, p + e, kind, a) - elastic.dstf(t, t0, p - e, kind, a)) / (2 * e)
        ana = theorem3.stf_second(t, t0, p, kind, wrt)
        assert np.max(np.abs(ana - num)) < 1e-6 * np.max(np.abs(ana)), wrt


@pytest.fixture(scope="module")
def problem():
    nx, nz, h = 40, 36, 16.0
    med = layered_medium(nz, h, [200.0], [2400.0, 2600.0], [2500.0, 3200.0], [1400.0, 1850.0])
    grid = Grid(nx, nz, h, 0.5 * h / med.vp_max(), 220)
    rec = np.array([5, 14, 20, 27, 33], dtype=np.int32)
    th_true = np.array([317.0, 420.0, 0.12, 9.0, 3e13, -2e13, 5e13])
    g = elastic.forward(grid, med, th_true, rec)
    sigma = 0.02 * np.abs(g).max()
    rng = np.random.default_rng(4)
    y = g + sigma * rng.standard_normal(g.shape)
    return grid, med, rec, th_true, y, sigma


def test_h1_plus_h2_is_the_misfit_hessian(problem):
    grid, med, rec, th_true, y, sigma = problem
    th = th_true * (1 + np.array([3e-3, -2e-3, 1e-2, -5e-3, 2e-2, 1e-2, -1e-2]))
    _, g, J = theorem3.data_gradient(grid, med, th, rec, y, sigma)
    H1 = laplace.hessian_h1(J, sigma)
    H2 = theorem3.hessian_h2(grid, med, th, rec, y, sigma)
    assert np.max(np.abs(H2)) > 1e-6 * np.max(np.abs(H1))
    s = np.sqrt(np.diag(H1))
    errs = []
    for rs in (1e-4, 5e-5):
        Hfd = np.empty((7, 7))
        for k in range(7):
            d = rs * abs(th[k])
            tp, tm = th.copy(), th.copy()
            tp[k] += d
            tm[k] -= d
            gp = theorem3.data_gradient(grid, med, tp, rec, y, sigma)[0]
            gm = theorem3.data_gradient(grid, med, tm, rec, y, sigma)[0]
            Hfd[:, k] = (gp - gm) / (2 * d)
        Hfd = 0.5 * (Hfd + Hfd.T)
        errs.append(np.max(np.abs((H1 + H2 - Hfd) / np.outer(s, s))))
    # the gap is the O(d^2) truncation of the differences (ratio 4 per
    # halving), far below the size of H_2 itself
    assert 3.5 < errs[0] / errs[1] < 4.5, errs
    assert errs[1] < 1e-6, errs
    assert np.max(np.abs(H2 / np.outer(s, s))) > 1e4 * errs[1]


def test_gauss_newton_reaches_a_stationary_point(problem):
    grid, med, rec, th_true, y, sigma = problem
    prior = laplace.uniform_prior(th_true * 0.5, th_true * 1.5 + 1.0)
    th_hat = theorem3.map_gauss_newton(grid, med, y, th_true, rec, sigma, prior, iters=6)
    grad, _, J = theorem3.data_gradient(grid, med, th_hat, rec, y, sigma)
    H1 = laplace.hessian_h1(J, sigma)
    s = np.sqrt(np.diag(H1))
    g0, _, _ = theorem3.data_gradient(grid, med, th_true, rec, y, sigma)
    assert np.max(np.abs(grad / s)) < 1e-8 * np.max(np.abs(g0 / s))
    # Theorem 1: theta^ - theta* is of the posterior's size
    assert np.max(np.abs((th_hat - th_true) * s)) < 6.0


def test_theorem3_exact_on_linear_gaussian_model():
    rng = np.random.default_rng(8)
    d, K, sigma = 3, 30, 0.5
    A = rng.standard_normal((K, d))
    Gamma = np.diag([0.7, 1.2, 0.4])
    prior = {"kind": "gaussian", "mean": np.zeros(d), "cov": Gamma}
    H1 = A.T @ A / sigma**2
    exact = 0.5 * np.linalg.slogdet(np.eye(d) + Gamma @ H1)[1]
    Hpost = H1 + np.linalg.inv(Gamma)
    vals = []
    for _ in range(20000):
        th = rng.multivariate_normal(np.zeros(d), Gamma)
        y = A @ th + sigma * rng.standard_normal(K)
        th_hat = np.linalg.solve(Hpost, A.T @ y / sigma**2)   # linear: MAP in closed form
        vals.append(theorem3.theorem3_integrand(H1, np.zeros((d, d)), th_hat, prior)[0])
    vals = np.array(vals)
    assert abs(vals.mean() - exact) < 4 * vals.std() / math.sqrt(len(vals)), (vals.mean(), exact)
