"""Pins of the oracle's finite-difference operator and leapfrog solve (CPU).

Section 3.3.1 names a second-order scheme built from D-, D+, D0 with a
traction-free top and the explicit central-difference time step.  The
oracle's operator is minus the gradient of a discrete elastic energy; these
tests pin it to closed forms (uniform strain energy, rigid rotation, exact
differentiation of quadratics), to symmetry, to reciprocity of the solve,
to exact discrete energy conservation and to second-order convergence of a
manufactured solution that includes the free surface.
"""
import ctypes
import math

import numpy as np
import pytest
import sympy as sp

from oracle import _clib, elastic
from synthetic import Grid, Medium


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def grad_energy(lam, mu, u, h):
    nz, nx = lam.shape
    g = np.zeros((2, nz, nx))
    u = np.ascontiguousarray(u, dtype=np.float64)
    _clib.lib().oracle_energy_gradient(nx, nz, h, _dp(np.ascontiguousarray(lam)),
                                       _dp(np.ascontiguousarray(mu)), _dp(u), _dp(g))
    return g


def apply_op(lam, mu, u, h):
    nz, nx = lam.shape
    out = np.zeros((2, nz, nx))
    u = np.ascontiguousarray(u, dtype=np.float64)
    _clib.lib().oracle_apply_operator(nx, nz, h, _dp(np.ascontiguousarray(lam)),
                                      _dp(np.ascontiguousarray(mu)), _dp(u), _dp(out))
    return out


def energy(lam, mu, u, h):
    # V is quadratic, so V(u) = 1/2 <u, grad V(u)>
    return 0.5 * float(np.sum(u * grad_energy(lam, mu, u, h)))


@pytest.mark.parametrize("nx,nz", [(9, 7), (16, 11)])
def test_uniform_strain_energy_closed_form(nx, nz):
    h, lam0, mu0 = 3.0, 2.3, 1.7
    lam = np.full((nz, nx), lam0)
    mu = np.full((nz, nx), mu0)
    z, x = np.meshgrid(np.arange(nz) * h, np.arange(nx) * h, indexing="ij")
    area = (nx - 1) * h * (nz - 1) * h
    for exx, ezz, exz in [(1e-3, 0, 0), (0, 2e-3, 0), (1e-3, -3e-3, 0),
                          (0, 0, 5e-4), (2e-4, 7e-4, -3e-4)]:
        # u = (exx x + exz z, exz x + ezz z): symmetric strain, no rotation
        u = np.stack([exx * x + exz * z, exz * x + ezz * z])
        w = 0.5 * lam0 * (exx + ezz) ** 2 + mu0 * (exx**2 + ezz**2 + 2 * exz**2)
        assert abs(energy(lam, mu, u, h) - w * area) < 1e-12 * max(w * area, 1e-20)


def test_rigid_motions_have_zero_energy():
    nx, nz, h = 12, 9, 2.0
    lam = np.full((nz, nx), 3.0)
    mu = np.full((nz, nx), 1.3)
    z, x = np.meshgrid(np.arange(nz) * h, np.arange(nx) * h, indexing="ij")
    for u in [np.stack([np.ones_like(x), 0 * x]), np.stack([0 * x, np.ones_like(x)]),
              np.stack([-z, x]) * 1e-3]:
        scale = 0.5 * 1.3 * float(np.sum(u**2))
        assert abs(energy(lam, mu, u, h)) < 1e-13 * max(scale, 1.0)


def test_interior_operator_exact_on_quadratics():
    # linear coefficients and quadratic displacements: every D+(a D-) and
    # D0(c D0) term differentiates exactly, so A_h u = div sigma(u) at nodes
    # away from the edges.
    nx, nz, h = 14, 12, 0.5
    X, Z = sp.symbols("x z")
    lam_e = 2.0 + 0.3 * X - 0.2 * Z
    mu_e = 1.0 + 0.1 * X + 0.25 * Z
    ue = 0.3 * X**2 - 0.2 * X * Z + 0.1 * Z**2 + X
    ve = -0.1 * X**2 + 0.4 * X * Z + 0.2 * Z**2 - Z
    exx, ezz, exz = sp.diff(ue, X), sp.diff(ve, Z), sp.diff(ue, Z) + sp.diff(ve, X)
    sxx = lam_e * (exx + ezz) + 2 * mu_e * exx
    szz = lam_e * (exx + ezz) + 2 * mu_e * ezz
    sxz = mu_e * exz
    divx = sp.diff(sxx, X) + sp.diff(sxz, Z)
    divz = sp.diff(sxz, X) + sp.diff(szz, Z)
    f = lambda e: sp.lambdify((X, Z), e, "numpy")  # noqa: E731
    z, x = np.meshgrid(np.arange(nz) * h, np.arange(nx) * h, indexing="ij")
    full = lambda e: np.broadcast_to(f(e)(x, z), x.shape).astype(float)  # noqa: E731
    lam, mu = full(lam_e), full(mu_e)
    u = np.stack([full(ue), full(ve)])
    A = apply_op(lam, mu, u, h)
    sl = (slice(2, nz - 2), slice(2, nx - 2))
    assert np.max(np.abs(A[0][sl] - full(divx)[sl])) < 1e-10
    assert np.max(np.abs(A[1][sl] - full(divz)[sl])) < 1e-10


def _random_medium(rng, nz, nx):
    lam = rng.uniform(1.0, 3.0, (nz, nx))
    mu = rng.uniform(0.5, 2.0, (nz, nx))
    rho = rng.uniform(1.0, 2.0, (nz, nx))
    return rho, lam, mu


def test_energy_hessian_symmetric_and_semidefinite():
    rng = np.random.default_rng(0)
    nx, nz, h = 7, 6, 1.5
    _, lam, mu = _random_medium(rng, nz, nx)
    n = 2 * nx * nz
    K = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        K[:, j] = grad_energy(lam, mu, e.reshape(2, nz, nx), h).ravel()
    assert np.max(np.abs(K - K.T)) < 1e-13 * np.max(np.abs(K))
    ev = np.linalg.eigvalsh(0.5 * (K + K.T))
    assert ev.min() > -1e-12 * ev.max()
    # With the rigid edges removed the operator is definite: A_h = -M^-1 K
    # has strictly negative eigenvalues on the free nodes.
    free = np.ones((2, nz, nx), bool)
    free[:, :, 0] = free[:, :, -1] = free[:, -1, :] = False
    idx = np.nonzero(free.ravel())[0]
    Kf = K[np.ix_(idx, idx)]
    assert np.linalg.eigvalsh(Kf).min() > 0


def test_solve_reciprocity():
    # M u'' = -K u + F with symmetric K and diagonal M: the response at A to
    # a unit load at B equals the response at B to a unit load at A.
    rng = np.random.default_rng(1)
    nx, nz, h = 20, 16, 10.0
    rho, lam, mu = _random_medium(rng, nz, nx)
    lam *= 1e9
    mu *= 1e9
    rho *= 1e3
    med = Medium("nodal", rho, lam, mu)
    vmax = float(np.max(np.sqrt((lam + 2 * mu) / rho)))
    grid = Grid(nx, nz, h, 0.5 * h / vmax, 120)
    S = np.sin(np.arange(grid.nsteps) * 0.3) * np.exp(-np.arange(grid.nsteps) / 40.0)
    A = (5, 0, 1)   # (i, k, component): a surface node, depth component
    B = (13, 9, 0)  # an interior node, x component

    def load(at):
        i, k, c = at
        W = np.zeros((2, 1, 1))
        wk = 0.5 if k == 0 else 1.0
        W[c, 0, 0] = 1.0 / (h * h * wk)   # unit nodal load F = h^2 w f
        return (i, k, W, S)

    trA = elastic.solve_terms(grid, med, [load(B)], [A[0]], [A[1]])[:, 0, A[2]]
    trB = elastic.solve_terms(grid, med, [load(A)], [B[0]], [B[1]])[:, 0, B[2]]
    assert np.max(np.abs(trA)) > 0
    assert np.max(np.abs(trA - trB)) < 1e-10 * np.max(np.abs(trA))


def test_leapfrog_conserves_discrete_energy():
    rng = np.random.default_rng(2)
    nx, nz, h = 24, 20, 5.0
    rho, lam, mu = _random_medium(rng, nz, nx)
    med = Medium("nodal", rho, lam, mu)
    vmax = float(np.max(np.sqrt((lam + 2 * mu) / rho)))
    dt = 0.5 * h / vmax
    z, x = np.meshgrid(np.arange(nz) * h, np.arange(nx) * h, indexing="ij")
    bump = np.exp(-(((x - 60) / 15) ** 2 + ((z - 30) / 15) ** 2))
    u0 = np.stack([bump, -0.5 * bump])
    u0[:, :, 0] = u0[:, :, -1] = u0[:, -1, :] = 0
    wts = np.ones((nz, nx))
    wts[0, :] *= 0.5
    mass = h * h * wts * rho

    def state(n):
        g = Grid(nx, nz, h, dt, n)
        _, fin = elastic.solve_terms(g, med, [], np.array([1], np.int32),
                                     u0=u0, um1=u0, want_final=True)
        return fin

    def E(n):
        a, b = state(n), state(n + 1)
        kin = 0.5 * np.sum(mass * (((b - a) / dt) ** 2).sum(axis=0))
        pot = 0.5 * float(np.sum(b * grad_energy(lam, mu, a, h)))
        return kin + pot

    e0 = E(0)
    for n in (50, 333, 2000):
        assert abs(E(n) - e0) < 1e-10 * e0


def _mms_error(n):
    L = 1000.0
    h = L / (n - 1)
    X, Z, T = sp.symbols("x z t")
    rho_e = 2000.0 + 300.0 * sp.sin(2 * X / L) * sp.cos(Z / L)
    lam_e = 8e9 * (1 + 0.2 * sp.cos(3 * X / L + Z / L))
    mu_e = 4e9 * (1 + 0.15 * sp.sin(X / L - 2 * Z / L))
    # vanishes on the rigid edges x = 0, x = L, z = L; free top z = 0
    Xu = sp.sin(sp.pi * X / L) * sp.cos(sp.pi * Z / (2 * L))
    Xv = sp.sin(2 * sp.pi * X / L) * sp.cos(sp.pi * Z / (2 * L)) * (1 + Z / L)
    om = 2 * sp.pi * 3.0
    Tt = sp.cos(om * T)
    exx, ezz, exz = sp.diff(Xu, X), sp.diff(Xv, Z), sp.diff(Xu, Z) + sp.diff(Xv, X)
    sxx = lam_e * (exx + ezz) + 2 * mu_e * exx
    szz = lam_e * (exx + ezz) + 2 * mu_e * ezz
    sxz = mu_e * exz
    divx = sp.diff(sxx, X) + sp.diff(sxz, Z)
    divz = sp.diff(sxz, X) + sp.diff(szz, Z)
    z, x = np.meshgrid(np.arange(n) * h, np.arange(n) * h, indexing="ij")
    ev = lambda e: np.broadcast_to(sp.lambdify((X, Z), e, "numpy")(x, z), x.shape).astype(float)  # noqa: E731
    rho, lam, mu = ev(rho_e), ev(lam_e), ev(mu_e)
    med = Medium("nodal", rho, lam, mu)
    vmax = float(np.max(np.sqrt((lam + 2 * mu) / rho)))
    tend = 0.12
    nsteps = int(math.ceil(tend / (0.4 * h / vmax)))
    dt = tend / nsteps
    grid = Grid(n, n, h, dt, nsteps)
    Xs = np.stack([ev(Xu), ev(Xv)])
    # f = rho u*_tt - div sigma(u*), plus the surface load (2/h) sigma(u*) n
    # with n = (0, -1) on the top row, all separable in time.
    W1 = rho * Xs
    W2 = -np.stack([ev(divx), ev(divz)])
    W2[0, 0, :] += (2.0 / h) * (-ev(sxz)[0, :])
    W2[1, 0, :] += (2.0 / h) * (-ev(szz)[0, :])
    tm = np.arange(nsteps) * dt
    Tf = sp.lambdify(T, Tt, "numpy")
    Tdd = sp.lambdify(T, sp.diff(Tt, T, 2), "numpy")
    terms = [(0, 0, W1, Tdd(tm)), (0, 0, W2, Tf(tm))]
    _, fin = elastic.solve_terms(grid, med, terms, np.array([1], np.int32),
                                 u0=Xs * Tf(0.0), um1=Xs * Tf(-dt), want_final=True)
    exact = Xs * Tf(tend)
    return np.max(np.abs(fin - exact)) / np.max(np.abs(exact))


def test_manufactured_solution_second_order():
    e = [_mms_error(n) for n in (17, 33, 65)]
    rates = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert e[-1] < 1e-2
    assert all(1.8 < r < 2.3 for r in rates), (e, rates)
