"""Oracle forward model: source discretisation, wavelets, FD solves, Jacobian.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain FP64.
"""
from __future__ import annotations

import ctypes
import math
from concurrent.futures import ThreadPoolExecutor
from typing import Optional, Sequence

import numpy as np

from . import _clib

NTHETA = 7


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


# ---------------------------------------------------------------------------
# Regularised Dirac delta and its derivative (Section 3.3.2, item 2, the
# fourth-order, twice continuously differentiable discretisations).
# ---------------------------------------------------------------------------
def delta_1d(alpha: float, h: float):
    """Weights of delta(x - x_s) on nodes k-2..k+3, where x_k <= x_s < x_{k+1}
    and alpha = (x_s - x_k)/h.  Returns an array of 6 values (units 1/h)."""
    a = alpha
    P = 5 * a**5 / 3 - 7 * a**6 / 24 - 17 * a**7 / 12 + 9 * a**8 / 8 - a**9 / 4
    d = np.array([
        a / 12 - a**2 / 24 - a**3 / 12 - 19 * a**4 / 24 + P,
        -2 * a / 3 + 2 * a**2 / 3 + a**3 / 6 + 4 * a**4 - 5 * P,
        1 - 5 * a**2 / 4 - 97 * a**4 / 12 + 10 * P,
        2 * a / 3 + 2 * a**2 / 3 - a**3 / 6 + 49 * a**4 / 6 - 10 * P,
        -a / 12 - a**2 / 24 + a**3 / 12 - 33 * a**4 / 8 + 5 * P,
        5 * a**4 / 6 - P,
    ])
    return d / h


def ddelta_1d(alpha: float, h: float):
    """Weights of delta'(x - x_s) on nodes k-2..k+3 (units 1/h^2)."""
    a = alpha
    R = -25 * a**4 / 12 - 3 * a**5 / 4 + 59 * a**6 / 12 - 4 * a**7 + a**8
    d = np.array([
        -1 / 12 + a / 12 + a**2 / 4 + 2 * a**3 / 3 + R,
        2 / 3 - 4 * a / 3 - a**2 / 2 - 7 * a**3 / 2 - 5 * R,
        5 * a / 2 + 22 * a**3 / 3 + 10 * R,
        -2 / 3 - 4 * a / 3 + a**2 / 2 - 23 * a**3 / 3 - 10 * R,
        1 / 12 + a / 12 - a**2 / 4 + 4 * a**3 + 5 * R,
        -5 * a**3 / 6 - R,
    ])
    return d / (h * h)


def locate(xs: float, h: float):
    """Node index k with x_k <= x_s < x_{k+1} and alpha = (x_s - x_k)/h."""
    k = int(math.floor(xs / h))
    return k, xs / h - k


def source_window(theta: Sequence[float], h: float):
    """Spatial part of f = S(t) M grad(delta(x - x_s)) (Section 2.1, point
    moment-tensor source), with grad(delta) the Cartesian product of the 1-D
    regularised delta and delta' (Section 3.3.2).

    Returns (i0, k0, W) with W[c][kk][ii] the force density (per unit S) on
    node (i0+ii, k0+kk), c = 0 (x) / 1 (depth).
    """
    xs, zs = theta[0], theta[1]
    mxx, mxz, mzz = theta[4], theta[5], theta[6]
    kx, ax = locate(xs, h)
    kz, az = locate(zs, h)
    dx, dpx = delta_1d(ax, h), ddelta_1d(ax, h)
    dz, dpz = delta_1d(az, h), ddelta_1d(az, h)
    # rows index depth (kk), columns index x (ii)
    gx = np.outer(dz, dpx)   # d/dx delta  = delta'(x) delta(z)
    gz = np.outer(dpz, dx)   # d/dz delta  = delta(x) delta'(z)
    W = np.empty((2, 6, 6))
    W[0] = mxx * gx + mxz * gz
    W[1] = mxz * gx + mzz * gz
    return kx - 2, kz - 2, W


# ---------------------------------------------------------------------------
# Source time functions.
# ---------------------------------------------------------------------------
def stf(t, t0: float, p: float, kind: str):
    """kind 'gauss': the paper's Gaussian (Section 4.1) with frequency
    parameter omega = p:  S = omega/sqrt(2 pi) exp(-omega^2 (t-t0)^2 / 2).
    kind 'gauss_deriv': time derivative of that Gaussian with omega = 2 pi p
    (p = f in Hz, the spectral peak of the wavelet)."""
    t = np.asarray(t, dtype=np.float64)
    if kind == "gauss":
        w = p
        return w / math.sqrt(2 * math.pi) * np.exp(-0.5 * w * w * (t - t0) ** 2)
    if kind == "gauss_deriv":
        w = 2 * math.pi * p
        g = w / math.sqrt(2 * math.pi) * np.exp(-0.5 * w * w * (t - t0) ** 2)
        return -w * w * (t - t0) * g
    raise ValueError(kind)


# ---------------------------------------------------------------------------
# Solves.
# ---------------------------------------------------------------------------
def _check_window(i0, k0, nx, nz, fw=6, fh=6):
    if i0 < 1 or k0 < 0 or i0 + fw > nx - 1 or k0 + fh > nz - 1:
        raise ValueError("source stencil touches a rigid edge or leaves the grid")


BC_CODES = {"rigid": 0, "absorbing": 1}


def solve_terms(grid, medium, terms, rec_i, rec_k=None, u0=None, um1=None,
                want_final=False):
    """Leapfrog solve driven by sum_q S_q(t_m) W_q.

    terms: list of (i0, k0, W[2][fh][fw], S[nsteps]); all W the same shape.
    Returns traces [nsteps+1][nrec][2] (and the final field [2][nz][nx])."""
    nx, nz = grid.nx, grid.nz
    rho, lam, mu = (np.ascontiguousarray(a, dtype=np.float64)
                    for a in medium.nodal(nx))
    rec_i = np.ascontiguousarray(rec_i, dtype=np.int32)
    rec_k = (np.zeros_like(rec_i) if rec_k is None
             else np.ascontiguousarray(rec_k, dtype=np.int32))
    nrec = rec_i.size
    nterm = len(terms)
    fh, fw = terms[0][2].shape[1:] if nterm else (1, 1)
    fi0 = np.array([t[0] for t in terms] or [0], dtype=np.int32)
    fk0 = np.array([t[1] for t in terms] or [0], dtype=np.int32)
    W = np.ascontiguousarray(np.stack([t[2] for t in terms]) if nterm
                             else np.zeros((1, 2, 1, 1)))
    S = np.ascontiguousarray(np.stack([np.asarray(t[3], dtype=np.float64)
                                       for t in terms]) if nterm
                             else np.zeros((1, max(grid.nsteps, 1))))
    traces = np.zeros((grid.nsteps + 1, nrec, 2))
    fin = np.zeros((2, nz, nx)) if want_final else None
    nul = ctypes.POINTER(ctypes.c_double)()
    u0c = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64)
    um1c = None if um1 is None else np.ascontiguousarray(um1, dtype=np.float64)
    rc = _clib.lib().oracle_solve(
        nx, nz, grid.h, grid.dt, grid.nsteps, _dp(rho), _dp(lam), _dp(mu),
        nterm, _ip(fi0), _ip(fk0), int(fw), int(fh), _dp(W), _dp(S),
        nrec, _ip(rec_i), _ip(rec_k), _dp(traces),
        nul if u0c is None else _dp(u0c), nul if um1c is None else _dp(um1c),
        _dp(fin) if want_final else nul, BC_CODES[getattr(grid, "bc", "rigid")])
    if rc != 0:
        raise ValueError("oracle_solve rejected its arguments")
    return (traces, fin) if want_final else traces


def forcing_term(grid, theta, stf_kind):
    i0, k0, W = source_window(theta, grid.h)
    _check_window(i0, k0, grid.nx, grid.nz)
    t = np.arange(grid.nsteps) * grid.dt
    return (i0, k0, W, stf(t, theta[2], theta[3], stf_kind))


def forward(grid, medium, theta, receivers, stf_kind="gauss_deriv"):
    """Receiver traces g_r(t_m; theta) (Section 2.2, parameter-to-observable
    map), shape [nsteps+1][nrec][2]."""
    return solve_terms(grid, medium, [forcing_term(grid, theta, stf_kind)],
                       receivers)


def fd_steps(theta, rel_step):
    return rel_step * np.abs(np.asarray(theta, dtype=np.float64))


def jacobian_literal(grid, medium, theta, receivers, rel_step=1e-4,
                     stf_kind="gauss_deriv", pool: Optional[ThreadPoolExecutor] = None):
    """Central-difference receiver Jacobian from 1 + 2*7 literal solves:
    J_j = (g(theta + d_j e_j) - g(theta - d_j e_j)) / (2 d_j), d_j = rel*|theta_j|.
    Returns (nominal traces, J[nsteps+1][nrec][2][7])."""
    theta = np.asarray(theta, dtype=np.float64)
    d = fd_steps(theta, rel_step)
    jobs = [theta]
    for j in range(NTHETA):
        for s in (+1.0, -1.0):
            tp = theta.copy()
            tp[j] += s * d[j]
            jobs.append(tp)
    run = lambda th: forward(grid, medium, th, receivers, stf_kind)  # noqa: E731
    res = list(pool.map(run, jobs)) if pool else [run(th) for th in jobs]
    nominal = res[0]
    J = np.empty(nominal.shape + (NTHETA,))
    for j in range(NTHETA):
        J[..., j] = (res[1 + 2 * j] - res[2 + 2 * j]) / (2 * d[j])
    return nominal, J


def deviation_terms(grid, theta, j, step, stf_kind):
    """Forcing F(theta + step e_j) - F(theta) as explicit terms (both windows
    kept separately, so no assumption on which factor changes)."""
    tp = np.asarray(theta, dtype=np.float64).copy()
    tp[j] += step
    a = forcing_term(grid, tp, stf_kind)
    b = forcing_term(grid, theta, stf_kind)
    return [a, (b[0], b[1], -b[2], b[3])]


def jacobian_deviation(grid, medium, theta, receivers, rel_step=1e-4,
                       stf_kind="gauss_deriv"):
    """The same central differences, but each perturbed solve is driven by
    the forcing difference F(theta +- d e_j) - F(theta); by linearity of the
    discrete solve it returns g(theta +- d e_j) - g(theta)."""
    theta = np.asarray(theta, dtype=np.float64)
    d = fd_steps(theta, rel_step)
    J = None
    for j in range(NTHETA):
        wp = solve_terms(grid, medium,
                         deviation_terms(grid, theta, j, d[j], stf_kind), receivers)
        wm = solve_terms(grid, medium,
                         deviation_terms(grid, theta, j, -d[j], stf_kind), receivers)
        if J is None:
            J = np.empty(wp.shape + (NTHETA,))
        J[..., j] = (wp - wm) / (2 * d[j])
    return J


def surface_nodes(nx):
    """All free (non-corner) surface nodes."""
    return np.arange(1, nx - 1, dtype=np.int32)


def noise_sigma(grid, medium, theta_bar, rel=1e-3, stf_kind="gauss_deriv"):
    """sigma = rel * peak |u| over all free surface nodes, both components and
    all recorded levels, for the nominal solve at the prior mean."""
    tr = forward(grid, medium, theta_bar, surface_nodes(grid.nx), stf_kind)
    return rel * float(np.max(np.abs(tr)))


# ---------------------------------------------------------------------------
# Forward sensitivities (Algorithm 1): solves driven by the
# derivative of the discretised source with respect to each parameter.
# ---------------------------------------------------------------------------
# The regularised delta / delta' weights as polynomials in alpha: per node
# offset -2..3 a printed base polynomial plus k_o times the common
# polynomial (P for delta, R for delta'), k = (1, -5, 10, -10, 5, -1).
_K = (1.0, -5.0, 10.0, -10.0, 5.0, -1.0)
_D_BASE = ((0, 1 / 12, -1 / 24, -1 / 12, -19 / 24), (0, -2 / 3, 2 / 3, 1 / 6, 4),
           (1, 0, -5 / 4, 0, -97 / 12), (0, 2 / 3, 2 / 3, -1 / 6, 49 / 6),
           (0, -1 / 12, -1 / 24, 1 / 12, -33 / 8), (0, 0, 0, 0, 5 / 6))
_D_COMMON = (0, 0, 0, 0, 0, 5 / 3, -7 / 24, -17 / 12, 9 / 8, -1 / 4)
_DP_BASE = ((-1 / 12, 1 / 12, 1 / 4, 2 / 3), (2 / 3, -4 / 3, -1 / 2, -7 / 2),
            (0, 5 / 2, 0, 22 / 3), (-2 / 3, -4 / 3, 1 / 2, -23 / 3),
            (1 / 12, 1 / 12, -1 / 4, 4), (0, 0, 0, -5 / 6))
_DP_COMMON = (0, 0, 0, 0, -25 / 12, -3 / 4, 59 / 12, -4, 1)


def weight_polys():
    """(delta polys times h, delta' polys times h^2), six numpy Polynomials
    each, coefficients in increasing powers of alpha."""
    P = np.polynomial.Polynomial
    d = [P(b) + k * P(_D_COMMON) for b, k in zip(_D_BASE, _K)]
    dp = [P(b) + k * P(_DP_COMMON) for b, k in zip(_DP_BASE, _K)]
    return d, dp


def dsource_window(theta: Sequence[float], h: float, j: int):
    """Derivative of the spatial source window with respect to x_s (j = 0)
    or z_s (j = 1): d/dx_s = (1/h) d/dalpha on that axis."""
    d_polys, dp_polys = weight_polys()
    xs, zs = theta[0], theta[1]
    mxx, mxz, mzz = theta[4], theta[5], theta[6]
    kx, ax = locate(xs, h)
    kz, az = locate(zs, h)
    ev = lambda ps, a, der: np.array([(p.deriv() if der else p)(a) for p in ps])  # noqa: E731
    dx, dpx = ev(d_polys, ax, j == 0) / h, ev(dp_polys, ax, j == 0) / h**2
    dz, dpz = ev(d_polys, az, j == 1) / h, ev(dp_polys, az, j == 1) / h**2
    if j == 0:
        dx, dpx = dx / h, dpx / h
    else:
        dz, dpz = dz / h, dpz / h
    gx = np.outer(dz, dpx)
    gz = np.outer(dpz, dx)
    W = np.empty((2, 6, 6))
    W[0] = mxx * gx + mxz * gz
    W[1] = mxz * gx + mzz * gz
    return kx - 2, kz - 2, W


def dstf(t, t0: float, p: float, kind: str, wrt: str):
    """Analytic derivative of stf with respect to t0 (wrt='t0') or to the
    frequency parameter (wrt='p')."""
    t = np.asarray(t, dtype=np.float64)
    tau = t - t0
    c = 1.0 / math.sqrt(2 * math.pi)
    if kind == "gauss":
        w = p
        e = np.exp(-0.5 * w * w * tau * tau)
        if wrt == "t0":
            return c * w**3 * tau * e
        return c * e * (1.0 - w * w * tau * tau)
    if kind == "gauss_deriv":
        w = 2 * math.pi * p
        e = np.exp(-0.5 * w * w * tau * tau)
        if wrt == "t0":
            return c * w * e * (w**2 - w**4 * tau * tau)
        # d/df = 2 pi d/domega of -c w^3 tau e
        return 2 * math.pi * c * e * (-3 * w**2 * tau + w**4 * tau**3)
    raise ValueError(kind)


def sensitivity_term(grid, theta, j, stf_kind):
    """Forcing d F / d theta_j as one separable term (window, series)."""
    theta = np.asarray(theta, dtype=np.float64)
    t = np.arange(grid.nsteps) * grid.dt
    if j in (0, 1):
        i0, k0, W = dsource_window(theta, grid.h, j)
        S = stf(t, theta[2], theta[3], stf_kind)
    elif j in (2, 3):
        i0, k0, W = source_window(theta, grid.h)
        S = dstf(t, theta[2], theta[3], stf_kind, "t0" if j == 2 else "p")
    else:
        unit = theta.copy()
        unit[4:] = 0.0
        unit[j] = 1.0
        i0, k0, W = source_window(unit, grid.h)
        S = stf(t, theta[2], theta[3], stf_kind)
    _check_window(i0, k0, grid.nx, grid.nz)
    return (i0, k0, W, S)


def jacobian_sensitivity(grid, medium, theta, receivers, stf_kind="gauss_deriv"):
    """Receiver Jacobian from 7 sensitivity solves: column j is the solve
    driven by dF/dtheta_j (the discrete scheme is linear in the forcing).
    Returns (nominal traces, J[nsteps+1][nrec][2][7])."""
    theta = np.asarray(theta, dtype=np.float64)
    nominal = forward(grid, medium, theta, receivers, stf_kind)
    J = np.empty(nominal.shape + (NTHETA,))
    for j in range(NTHETA):
        J[..., j] = solve_terms(grid, medium, [sensitivity_term(grid, theta, j, stf_kind)],
                                receivers)
    return nominal, J
