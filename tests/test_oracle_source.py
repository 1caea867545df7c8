"""Pins of the oracle's source discretisation and wavelets (CPU only).

The regularised delta and delta' (Section 3.3.2, item 2) are defined by
discrete moment conditions for polynomials up to degree four and by being
twice continuously differentiable in the source position; both are checked
here independently of the printed coefficient formulas.
"""
import math

import numpy as np
import pytest

from oracle import elastic

H = 7.0
ALPHAS = np.linspace(0.0, 0.999, 37)


@pytest.mark.parametrize("alpha", ALPHAS)
def test_delta_moment_conditions(alpha):
    # nodes k-2..k+3 relative to x_s: (o - alpha) h
    xs_rel = (np.arange(-2, 4) - alpha) * H
    d = elastic.delta_1d(alpha, H)
    dp = elastic.ddelta_1d(alpha, H)
    for p in range(5):
        mom = H * np.sum(d * xs_rel**p)
        assert abs(mom - (1.0 if p == 0 else 0.0)) < 1e-12 * max(1.0, H**p)
        # int phi delta'(x - xs) = -phi'(xs): for phi = (x-xs)^p only p=1 survives
        momp = H * np.sum(dp * xs_rel**p)
        assert abs(momp - (-1.0 if p == 1 else 0.0)) < 1e-12 * max(1.0, H**p) / H
    # degree 5 is not reproduced (the discretisation is exactly fourth order)
    assert abs(H * np.sum(d * xs_rel**5)) > 1e-6 * H**5 or alpha in (0.0,)


def _node_weight_poly(fn, offset):
    """Polynomial (in alpha) giving the weight of node k+offset."""
    a = np.linspace(0, 1, 25)
    vals = np.array([fn(x, 1.0)[offset + 2] for x in a])
    return np.polynomial.Polynomial.fit(a, vals, 10).convert()


@pytest.mark.parametrize("fn", [elastic.delta_1d, elastic.ddelta_1d])
def test_delta_twice_continuously_differentiable(fn):
    # A fixed node k+o receives weight w_o(alpha) while x_s is in cell k and
    # w_{o-1}(alpha - 1) once x_s moves into cell k+1.  C^2 in x_s means the
    # values and first two alpha-derivatives agree at alpha = 1 / 0.
    polys = {o: _node_weight_poly(fn, o) for o in range(-2, 4)}
    zero = np.polynomial.Polynomial([0.0])
    for o in range(-2, 5):
        left = polys.get(o, zero)       # cell k at alpha -> 1
        right = polys.get(o - 1, zero)  # cell k+1 at alpha -> 0
        for der in range(3):
            lv = left.deriv(der)(1.0) if der else left(1.0)
            rv = right.deriv(der)(0.0) if der else right(0.0)
            assert abs(lv - rv) < 1e-8, (o, der, lv, rv)


def test_source_window_is_moment_tensor_times_grad_delta():
    # Discrete analogue of int phi . M grad(delta) = -M : grad(phi)(x_s) for a
    # linear vector field phi = B x: the window must return -trace(M B^T).
    theta = np.array([503.3, 411.7, 0.2, 7.0, 1.3, -0.7, 2.1])
    i0, k0, W = elastic.source_window(theta, H)
    ii, kk = np.meshgrid(np.arange(6) + i0, np.arange(6) + k0)
    x, z = ii * H, kk * H
    M = np.array([[theta[4], theta[5]], [theta[5], theta[6]]])
    rng = np.random.default_rng(3)
    for _ in range(4):
        B = rng.standard_normal((2, 2))
        b = rng.standard_normal(2)
        phi = [B[0, 0] * x + B[0, 1] * z + b[0], B[1, 0] * x + B[1, 1] * z + b[1]]
        pair = H * H * (np.sum(W[0] * phi[0]) + np.sum(W[1] * phi[1]))
        assert abs(pair - (-np.sum(M * B))) < 1e-9 * np.abs(M).max()


def test_gauss_wavelet_closed_forms():
    t = np.linspace(-1, 3, 4001)
    t0, w = 1.1, 4.0
    g = elastic.stf(t, t0, w, "gauss")
    # unit area Gaussian with peak w/sqrt(2 pi) at t0
    assert abs(np.trapezoid(g, t) - 1.0) < 1e-9
    assert abs(g.max() - w / math.sqrt(2 * math.pi)) < 1e-6
    # gauss_deriv is the time derivative of the Gaussian with omega = 2 pi f
    f = 0.9
    gd = elastic.stf(t, t0, f, "gauss_deriv")
    G = elastic.stf(t, t0, 2 * math.pi * f, "gauss")
    num = np.gradient(G, t, edge_order=2)
    assert np.max(np.abs(gd - num)) < 1e-4 * np.max(np.abs(gd))


def test_weight_polynomial_tables_equal_printed_formulas():
    d_polys, dp_polys = elastic.weight_polys()
    for a in np.linspace(0, 0.999, 23):
        assert np.max(np.abs(np.array([p(a) for p in d_polys]) - elastic.delta_1d(a, 1.0))) < 1e-14
        assert np.max(np.abs(np.array([p(a) for p in dp_polys]) - elastic.ddelta_1d(a, 1.0))) < 1e-14


@pytest.mark.parametrize("alpha", [0.0, 0.13, 0.5, 0.77, 0.999])
def test_weight_derivatives_by_differentiated_moments(alpha):
    # d/dx_s of sum_j w_j(x_s) (x_j - x_s)^p h = const gives
    # sum_j w_j' (x_j - x_s)^p h = p sum_j w_j (x_j - x_s)^(p-1) h
    d_polys, dp_polys = elastic.weight_polys()
    xs_rel = (np.arange(-2, 4) - alpha) * H
    for polys, scale in ((d_polys, 1 / H), (dp_polys, 1 / H**2)):
        w = np.array([p(alpha) for p in polys]) * scale
        dw = np.array([p.deriv()(alpha) for p in polys]) * scale / H   # d/dx_s
        for p in range(1, 5):
            lhs = H * np.sum(dw * xs_rel**p)
            rhs = p * H * np.sum(w * xs_rel ** (p - 1))
            assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(rhs)), (p, lhs, rhs)
        assert abs(H * np.sum(dw)) < 1e-10 * np.max(np.abs(dw)) * H


@pytest.mark.parametrize("kind,p", [("gauss", 6.0), ("gauss_deriv", 7.5)])
def test_wavelet_derivatives_match_differences(kind, p):
    t = np.linspace(0, 1.2, 601)
    t0 = 0.4
    e = 1e-6
    num_t0 = (elastic.stf(t, t0 + e, p, kind) - elastic.stf(t, t0 - e, p, kind)) / (2 * e)
    num_p = (elastic.stf(t, t0, p + e, kind) - elastic.stf(t, t0, p - e, kind)) / (2 * e)
    a_t0 = elastic.dstf(t, t0, p, kind, "t0")
    a_p = elastic.dstf(t, t0, p, kind, "p")
    assert np.max(np.abs(a_t0 - num_t0)) < 1e-6 * np.max(np.abs(a_t0))
    assert np.max(np.abs(a_p - num_p)) < 1e-6 * np.max(np.abs(a_p))
