"""Oracle pieces of the Theorem-3 estimator (TEST INFRASTRUCTURE ONLY).

Theorem 3 evaluates, at the maximum a posteriori point theta^ of one data
set y = g(theta*) + eps,
    -1/2 log((2 pi)^N |H^-1|) - N/2 - h(theta^) - 1/2 tr(H^-1 grad grad h),
with H = H_1 + H_2 - grad grad h (eqs. for H, H_1 and H_2 in Theorem 2),
    H_2 = - sum_{r,m} grad grad g_r(t_m, theta^) o C_eps^-1 (y_r(t_m) - g_r(t_m, theta^)).
Here grad grad g comes straight from its definition: the solve is linear in
its forcing, so d^2 g / d theta_j d theta_k is the solve driven by
d^2 F / d theta_j d theta_k, the second derivative of the discretised point
source (the C^2 regularised delta/delta' weights of Section 3.3.2 item 2 and
the wavelet).  Moments enter F linearly, so pairs of moments vanish: 22
solves per sample.  The MAP point is found by Gauss-Newton steps with the
Jacobian of the forward-sensitivity solves (Algorithm 1).  Plain FP64.
"""
from __future__ import annotations

import math

import numpy as np

from . import elastic

SPATIAL = (0, 1)
TEMPORAL = (2, 3)
MOMENTS = (4, 5, 6)


def window_derivative(theta, h: float, ox: int, oz: int, moments=None):
    """d^(ox+oz) / dx_s^ox dz_s^oz of the source window M grad(delta) (both
    components), with the moment tensor of theta or the given (mxx, mxz, mzz)."""
    d_polys, dp_polys = elastic.weight_polys()
    kx, ax = elastic.locate(theta[0], h)
    kz, az = elastic.locate(theta[1], h)
    ev = lambda ps, a, o: np.array([p.deriv(o)(a) if o else p(a) for p in ps])  # noqa: E731
    dx = ev(d_polys, ax, ox) / h / h**ox
    dpx = ev(dp_polys, ax, ox) / h**2 / h**ox
    dz = ev(d_polys, az, oz) / h / h**oz
    dpz = ev(dp_polys, az, oz) / h**2 / h**oz
    mxx, mxz, mzz = theta[4:7] if moments is None else moments
    gx = np.outer(dz, dpx)      # delta'(x) delta(z)
    gz = np.outer(dpz, dx)      # delta(x) delta'(z)
    W = np.empty((2, 6, 6))
    W[0] = mxx * gx + mxz * gz
    W[1] = mxz * gx + mzz * gz
    return kx - 2, kz - 2, W


def stf_second(t, t0: float, p: float, kind: str, wrt: str):
    """Second derivatives of the wavelet: wrt in ('t0t0', 't0p', 'pp'), p the
    Gaussian's omega or the Gaussian derivative's frequency f."""
    t = np.asarray(t, dtype=np.float64)
    tau = t - t0
    c = 1.0 / math.sqrt(2 * math.pi)
    if kind == "gauss":
        w = p
        e = np.exp(-0.5 * w * w * tau * tau)
        if wrt == "t0t0":
            return c * w**3 * e * (w * w * tau * tau - 1.0)
        if wrt == "t0p":
            return c * w * w * tau * e * (3.0 - w * w * tau * tau)
        return c * w * tau * tau * e * (w * w * tau * tau - 3.0)
    if kind == "gauss_deriv":
        w = 2 * math.pi * p
        e = np.exp(-0.5 * w * w * tau * tau)
        if wrt == "t0t0":
            return c * w**5 * tau * e * (3.0 - w * w * tau * tau)
        if wrt == "t0p":   # d/df = 2 pi d/domega
            return 2 * math.pi * c * w * w * e * (w**4 * tau**4 - 6 * w * w * tau * tau + 3.0)
        return (4 * math.pi**2) * c * w * tau * e * (-(w * tau) ** 4 + 7 * (w * tau) ** 2 - 6.0)
    raise ValueError(kind)


def _unit_moment(j):
    m = [0.0, 0.0, 0.0]
    m[j - 4] = 1.0
    return m


def second_forcing_term(grid, theta, j: int, k: int, stf_kind: str):
    """d^2 F / d theta_j d theta_k as one separable (window, series) term, or
    None where it vanishes (two moments)."""
    theta = np.asarray(theta, dtype=np.float64)
    t = np.arange(grid.nsteps) * grid.dt
    t0, p = theta[2], theta[3]
    pair = sorted((j, k))
    a, b = pair
    if a in MOMENTS and b in MOMENTS:
        return None
    tname = {2: "t0", 3: "p"}
    if a in SPATIAL and b in SPATIAL:
        ox = (a == 0) + (b == 0)
        i0, k0, W = window_derivative(theta, grid.h, ox, 2 - ox)
        S = elastic.stf(t, t0, p, stf_kind)
    elif a in SPATIAL and b in TEMPORAL:
        i0, k0, W = window_derivative(theta, grid.h, int(a == 0), int(a == 1))
        S = elastic.dstf(t, t0, p, stf_kind, tname[b])
    elif a in TEMPORAL and b in TEMPORAL:
        i0, k0, W = window_derivative(theta, grid.h, 0, 0)
        S = stf_second(t, t0, p, stf_kind, tname[a] + tname[b])
    elif a in SPATIAL and b in MOMENTS:
        i0, k0, W = window_derivative(theta, grid.h, int(a == 0), int(a == 1), _unit_moment(b))
        S = elastic.stf(t, t0, p, stf_kind)
    else:  # temporal x moment
        i0, k0, W = window_derivative(theta, grid.h, 0, 0, _unit_moment(b))
        S = elastic.dstf(t, t0, p, stf_kind, tname[a])
    return (i0, k0, W, S)


def hessian_h2(grid, medium, theta, receivers, y, sigma: float, stf_kind="gauss_deriv"):
    """H_2 at theta for data y [nt][nrec][2] (Theorem 2), from the 22
    second-derivative solves."""
    g = elastic.forward(grid, medium, theta, receivers, stf_kind)
    r = (np.asarray(y, dtype=np.float64) - g) / (sigma * sigma)
    H2 = np.zeros((7, 7))
    for j in range(7):
        for k in range(j, 7):
            term = second_forcing_term(grid, theta, j, k, stf_kind)
            if term is None:
                continue
            D = elastic.solve_terms(grid, medium, [term], receivers)
            H2[j, k] = H2[k, j] = -float(np.sum(D * r))
    return H2


def data_gradient(grid, medium, theta, receivers, y, sigma: float, stf_kind="gauss_deriv"):
    """Gradient of 1/2 sum |y - g(theta)|^2 / sigma^2, and (g, J)."""
    g, J = elastic.jacobian_sensitivity(grid, medium, theta, receivers, stf_kind)
    r = (np.asarray(y, dtype=np.float64) - g) / (sigma * sigma)
    grad = -(J.reshape(-1, J.shape[-1]).T @ r.reshape(-1))
    return grad, g, J


def _prior_grad_hess(theta, prior):
    if prior["kind"] == "uniform":
        return np.zeros(7), np.zeros((7, 7))
    ci = np.linalg.inv(np.asarray(prior["cov"]))
    return -ci @ (np.asarray(theta) - np.asarray(prior["mean"])), -ci


def map_gauss_newton(grid, medium, y, theta0, receivers, sigma: float, prior: dict,
                     stf_kind="gauss_deriv", iters: int = 6):
    """theta^ = argmin 1/2 sum |y - g|^2/sigma^2 - h(theta) by Gauss-Newton
    steps (H_1 - grad grad h) dtheta = -(grad of the data term) + grad h,
    solved through the diagonal scaling of Section 3.3.3."""
    th = np.asarray(theta0, dtype=np.float64).copy()
    for _ in range(iters):
        grad, _, J = data_gradient(grid, medium, th, receivers, y, sigma, stf_kind)
        gh, Hh = _prior_grad_hess(th, prior)
        Jf = J.reshape(-1, J.shape[-1])
        H = (Jf.T @ Jf) / (sigma * sigma) - Hh
        rhs = -grad + gh
        s = np.sqrt(np.diag(H))
        step = np.linalg.solve(H / np.outer(s, s), rhs / s) / s
        th = th + step
    return th


def theorem3_integrand(H1, H2, theta_hat, prior: dict):
    """The bracket of Theorem 3 at theta^; returns (value, ok)."""
    _, Hh = _prior_grad_hess(theta_hat, prior)
    H = H1 + H2 - Hh
    n = H.shape[0]
    ld, ok = laplace_logdet(H)
    if not ok:
        return float("nan"), False
    tr = float(np.trace(np.linalg.solve(H, Hh)))
    from .laplace import log_prior
    return (-0.5 * (n * math.log(2 * math.pi) - ld) - 0.5 * n - log_prior(theta_hat, prior)
            - 0.5 * tr), True


def laplace_logdet(H):
    from .laplace import logdet_scaled
    return logdet_scaled(H)


def sample_terms(grid, medium, receivers, theta_star, noise, sigma: float, prior: dict,
                 stf_kind="gauss_deriv", iters: int = 6):
    """One outer sample of the Theorem-3 estimator: data y = g(theta*) +
    sigma * noise, theta^ by Gauss-Newton from theta*, H_1 and H_2 at theta^,
    and the integrand.  Returns a dict."""
    g = elastic.forward(grid, medium, theta_star, receivers, stf_kind)
    y = g + sigma * np.asarray(noise, dtype=np.float64).reshape(g.shape)
    th_hat = map_gauss_newton(grid, medium, y, theta_star, receivers, sigma, prior,
                              stf_kind, iters)
    _, _, J = data_gradient(grid, medium, th_hat, receivers, y, sigma, stf_kind)
    Jf = J.reshape(-1, J.shape[-1])
    H1 = (Jf.T @ Jf) / (sigma * sigma)
    H2 = hessian_h2(grid, medium, th_hat, receivers, y, sigma, stf_kind)
    val, ok = theorem3_integrand(H1, H2, th_hat, prior)
    return {"y": y, "theta_hat": th_hat, "H1": H1, "H2": H2, "value": val, "ok": ok}
