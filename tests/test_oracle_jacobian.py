"""Pins of the oracle's source-parameter Jacobian and Gauss-Newton Hessian.

The discrete solve is linear in the forcing, invariant under time shifts of
the wavelet and, in a homogeneous medium before edge reflections, under
horizontal shifts by whole cells; the central-difference Jacobian and H_1
(Theorem 2) inherit exact properties from that.
"""
import math

import numpy as np
import pytest

from oracle import elastic, laplace
from synthetic import Grid, homogeneous_medium, layered_medium


@pytest.fixture(scope="module")
def small():
    nx, nz, h = 40, 36, 16.0
    med = layered_medium(nz, h, [200.0], [2400.0, 2600.0], [2500.0, 3200.0],
                         [1400.0, 1850.0])
    grid = Grid(nx, nz, h, 0.5 * h / med.vp_max(), 220)
    rec = np.array([5, 14, 20, 27, 33], dtype=np.int32)
    theta = np.array([317.0, 420.0, 0.12, 9.0, 3e13, -2e13, 5e13])
    return grid, med, rec, theta


def test_superposition_in_moment_tensor(small):
    grid, med, rec, theta = small
    parts = []
    for j in (4, 5, 6):
        th = theta.copy()
        th[4:] = 0.0
        th[j] = theta[j]
        parts.append(elastic.forward(grid, med, th, rec))
    full = elastic.forward(grid, med, theta, rec)
    assert np.max(np.abs(full - sum(parts))) < 1e-12 * np.max(np.abs(full))


def test_moment_columns_equal_unit_moment_solves(small):
    grid, med, rec, theta = small
    _, J = elastic.jacobian_literal(grid, med, theta, rec)
    for j in (4, 5, 6):
        th = theta.copy()
        th[4:] = 0.0
        th[j] = 1.0
        unit = elastic.forward(grid, med, th, rec)
        err = np.max(np.abs(J[..., j] - unit)) / np.max(np.abs(unit))
        assert err < 1e-8


def test_time_shift_by_one_step(small):
    grid, med, rec, theta = small
    th = theta.copy()
    th[2], th[3] = 0.5, 8.0          # S(t <= 0) ~ exp(-(2 pi 8 0.5)^2/2) ~ 0
    a = elastic.forward(grid, med, th, rec)
    th2 = th.copy()
    th2[2] = th[2] + grid.dt
    b = elastic.forward(grid, med, th2, rec)
    assert np.max(np.abs(b[1:] - a[:-1])) < 1e-12 * np.max(np.abs(a))


def test_horizontal_translation_by_whole_cells():
    nx, nz, h = 64, 48, 16.0
    med = homogeneous_medium(nz, 2500.0, 3000.0, 1730.0)
    grid = Grid(nx, nz, h, 0.5 * h / med.vp_max(), 14)
    theta = np.array([30 * h + 5.0, 24 * h + 3.0, 0.01, 25.0, 1e13, 2e13, 3e13])
    rec_i = np.array([26, 30, 34], dtype=np.int32)
    rec_k = np.array([20, 27, 24], dtype=np.int32)
    a = elastic.solve_terms(grid, med, [elastic.forcing_term(grid, theta, "gauss_deriv")],
                            rec_i, rec_k)
    th2 = theta.copy()
    th2[0] += 3 * h
    b = elastic.solve_terms(grid, med, [elastic.forcing_term(grid, th2, "gauss_deriv")],
                            rec_i + 3, rec_k)
    assert np.max(np.abs(a)) > 0
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(a))


def test_deviation_forcing_matches_literal_differences(small):
    grid, med, rec, theta = small
    _, J = elastic.jacobian_literal(grid, med, theta, rec)
    Jd = elastic.jacobian_deviation(grid, med, theta, rec)
    for j in range(7):
        err = np.linalg.norm(Jd[..., j] - J[..., j]) / np.linalg.norm(J[..., j])
        assert err < 1e-9, (j, err)


def test_central_difference_truncation_is_second_order(small):
    grid, med, rec, theta = small
    _, J1 = elastic.jacobian_literal(grid, med, theta, rec, rel_step=2e-3)
    _, J2 = elastic.jacobian_literal(grid, med, theta, rec, rel_step=1e-3)
    _, J4 = elastic.jacobian_literal(grid, med, theta, rec, rel_step=5e-4)
    for j in (0, 1, 2, 3):
        e1 = np.linalg.norm(J1[..., j] - J2[..., j])
        e2 = np.linalg.norm(J2[..., j] - J4[..., j])
        assert 3.0 < e1 / e2 < 5.0, (j, e1 / e2)


def test_h1_properties(small):
    grid, med, rec, theta = small
    _, J = elastic.jacobian_literal(grid, med, theta, rec)
    sigma = 0.37
    H = laplace.hessian_h1(J, sigma)
    Hr = laplace.hessian_h1_per_receiver(J, sigma)
    assert np.max(np.abs(H - H.T)) == 0.0
    assert np.max(np.abs(Hr.sum(axis=0) - H)) < 1e-12 * np.max(np.abs(H))
    ld, ok = laplace.logdet_scaled(H)
    assert ok and np.isfinite(ld)
    H2 = laplace.hessian_h1(J, 2 * sigma)
    assert np.max(np.abs(4 * H2 - H)) < 1e-14 * np.max(np.abs(H))
    # additive over time windows as well as receivers
    Ha = laplace.hessian_h1(J[:100], sigma)
    Hb = laplace.hessian_h1(J[100:], sigma)
    assert np.max(np.abs(Ha + Hb - H)) < 1e-12 * np.max(np.abs(H))


def test_scaling_moments_adds_four_log_c(small):
    # u is linear in M: scaling M by c scales the x, z, t0, f columns of J by c
    # and leaves the M columns unchanged, so det H_1 grows by c^8 and D^_KL by
    # 4 log c (uniform prior, fixed sigma).
    grid, med, rec, theta = small
    lo = np.array([100, 300, 0.1, 5, 1e13, -5e13, 1e13])
    hi = np.array([500, 500, 0.3, 10, 1e14, 5e13, 1e14])
    prior = laplace.uniform_prior(lo, hi)
    c = 2.5
    th2 = theta.copy()
    th2[4:] *= c
    v = []
    for th in (theta, th2):
        _, J = elastic.jacobian_literal(grid, med, th, rec)
        v.append(laplace.dkl_hat(laplace.hessian_h1(J, 0.1), th, prior)[0])
    assert abs(v[1] - v[0] - 4 * math.log(c)) < 1e-7


def test_sensitivity_jacobian_matches_central_differences(small):
    # Algorithm 1's sensitivity solves (driven by dF/dtheta_j) against the
    # central differences: equal up to the O(d^2) truncation of the latter
    grid, med, rec, theta = small
    nom_s, Js = elastic.jacobian_sensitivity(grid, med, theta, rec)
    nom_c, Jc = elastic.jacobian_literal(grid, med, theta, rec, rel_step=1e-4)
    _, Jc2 = elastic.jacobian_literal(grid, med, theta, rec, rel_step=5e-5)
    assert np.array_equal(nom_s, nom_c)
    for j in range(7):
        n = np.linalg.norm(Js[..., j])
        e1 = np.linalg.norm(Js[..., j] - Jc[..., j]) / n
        e2 = np.linalg.norm(Js[..., j] - Jc2[..., j]) / n
        assert e2 < 2e-6, (j, e2)
        if j < 4:   # nonlinear parameters: the gap is the O(d^2) truncation
            assert 3.5 < e1 / e2 < 4.5, (j, e1, e2)
        else:       # linear in the moments: exact up to rounding
            assert e2 < 1e-9, (j, e2)


def test_pipeline_dkl_same_from_either_jacobian():
    # the two Jacobians of Algorithm 1 (central differences, sensitivity
    # solves) give the same D^_KL up to the O(d^2) truncation of the former
    import synthetic
    from oracle import pipeline
    wl = synthetic.config("c1", nsample=4, grid_override=(48, 40, 160))[0]
    a = pipeline.query(wl, sigma=0.01, jacobian="fd")
    b = pipeline.query(wl, sigma=0.01, jacobian="sensitivity")
    assert np.max(np.abs(a["dkl"] - b["dkl"])) < 1e-4
    assert np.array_equal(a["nominal"], b["nominal"])


def test_hessian_grows_with_receivers_and_recording_time():
    # the paper's concentration argument: H_1 is O(N), N = N_R x N_t.  In the
    # closed rigid box the signal persists, and on a dense surface array
    # doubling the receivers or the record length doubles H_1, so D^_KL
    # gains N_theta/2 log 2 (log det H_1 grows by 7 log 2) -- here within 15 %
    import synthetic
    wl = synthetic.config("c1", nsample=1, grid_override=(64, 64, 1600))[0]
    rec = np.arange(1, 63, dtype=np.int32)
    th = wl.theta[0]
    _, J = elastic.jacobian_sensitivity(wl.grid, wl.medium, th, rec, wl.stf)
    sig = 1e-3 * np.abs(elastic.forward(wl.grid, wl.medium, th, rec, wl.stf)).max()
    prior = laplace.uniform_prior(wl.lo, wl.hi)
    dkl = lambda JJ: laplace.dkl_hat(laplace.hessian_h1(JJ, sig), th, prior)[0]  # noqa: E731
    # recording time: windows [0, 800] and [0, 1600] steps (H_1 additive in time)
    gain_t = dkl(J) - dkl(J[:801])
    assert abs(gain_t / (3.5 * math.log(1601 / 801)) - 1) < 0.15, gain_t
    # receivers: every second surface node against all of them
    half = np.arange(0, 62, 2)
    gain_r = dkl(J) - dkl(J[:, half])
    assert abs(gain_r / (3.5 * math.log(62 / 31)) - 1) < 0.15, gain_r
    # and H_1 itself doubles: scaled trace of the sub-array's H_1 is half
    Hf = laplace.hessian_h1(J, sig)
    ratio = np.trace(Hf / np.diag(Hf)[None, :]) / np.trace(
        laplace.hessian_h1(J[:, half], sig) / np.diag(Hf)[None, :])
    assert abs(ratio / 2 - 1) < 0.15, ratio
