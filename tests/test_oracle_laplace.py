"""Pins of the oracle's Laplace estimator, averages and design search (CPU).

Closed forms used: the KL divergence of a Gaussian posterior against a
uniform prior; the exact expected information gain of a linear-Gaussian
model; log-determinants from a symmetric eigen-decomposition.
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import laplace, smolyak

N = 7


def _spd(rng, scales):
    A = rng.standard_normal((N, N))
    C = A @ A.T + N * np.eye(N)
    D = np.diag(scales)
    return D @ C @ D


def test_scaled_logdet_matches_eigendecomposition():
    rng = np.random.default_rng(0)
    scales = np.array([1e-4, 1e-4, 1.0, 10.0, 1e-14, 1e-14, 1e-14])
    for _ in range(20):
        H = _spd(rng, scales * rng.uniform(0.5, 2, N))
        ld, ok = laplace.logdet_scaled(H)
        s = np.sqrt(np.diag(H))
        ref = np.sum(np.log(np.linalg.eigvalsh(H / np.outer(s, s)))) + 2 * np.sum(np.log(s))
        assert ok and abs(ld - ref) < 1e-12 * max(1, abs(ref))


def test_not_positive_definite_is_flagged():
    H = np.eye(N)
    H[0, 1] = H[1, 0] = 1.5
    assert not laplace.logdet_scaled(H)[1]
    H = np.eye(N)
    H[3, 3] = -1
    assert not laplace.logdet_scaled(H)[1]
    H = np.eye(N)
    H[2, 2] = np.nan
    assert not laplace.logdet_scaled(H)[1]


def test_uniform_prior_diagonal_closed_form():
    # Posterior N(theta*, H^-1) with diagonal H against a uniform box: the KL
    # divergence is sum_j log(b_j - a_j) - 1/2 log(2 pi e / H_jj).
    rng = np.random.default_rng(1)
    lo = rng.uniform(-5, 0, N)
    hi = lo + rng.uniform(0.5, 20, N)
    Hd = rng.uniform(0.1, 1e6, N)
    v, ok = laplace.dkl_hat(np.diag(Hd), 0.5 * (lo + hi), laplace.uniform_prior(lo, hi))
    ref = np.sum(np.log(hi - lo) - 0.5 * np.log(2 * math.pi * math.e / Hd))
    assert ok and abs(v - ref) < 1e-12 * abs(ref)


def test_reparametrisation_invariance():
    rng = np.random.default_rng(2)
    lo = np.array([80, 630, 0.1, 5, 1e13, 1e13, 1e13])
    hi = np.array([1180, 1180, 0.3, 10, 1e14, 1e14, 1e14])
    H = _spd(rng, 1.0 / (hi - lo))
    th = 0.5 * (lo + hi)
    D = rng.uniform(0.1, 10, N)
    v0, _ = laplace.dkl_hat(H, th, laplace.uniform_prior(lo, hi))
    Hs = H / np.outer(D, D)   # theta' = D theta
    v1, _ = laplace.dkl_hat(Hs, D * th, laplace.uniform_prior(D * lo, D * hi))
    assert abs(v0 - v1) < 1e-11 * abs(v0)


def _linear_gaussian(rng, n_meas):
    G = rng.standard_normal((n_meas, N))
    sigma = 0.3
    H1 = G.T @ G / sigma**2
    L = np.tril(rng.standard_normal((N, N))) + 3 * np.eye(N)
    Gam = L @ L.T
    mu = rng.standard_normal(N)
    return H1, Gam, mu


def _sigma_points(mu, Gam):
    # 2N points with equal weights reproduce mean and covariance exactly
    L = np.linalg.cholesky(Gam)
    pts = [mu + s * math.sqrt(N) * L[:, j] for j in range(N) for s in (1, -1)]
    return np.array(pts), np.full(2 * N, 1.0 / (2 * N))


def test_linear_gaussian_laplace_estimate_and_gap():
    # g = G theta: H_1 is constant, h is quadratic, so the prior average of
    # D^_KL is exact on a rule that integrates quadratics: 1/2 log det(Gam H_1).
    # The exact EIG is 1/2 log det(I + Gam H_1); the gap is O(1/N).
    rng = np.random.default_rng(3)
    gaps = []
    for n_meas in (40, 400, 4000):
        H1, Gam, mu = _linear_gaussian(np.random.default_rng(3), 40)
        H1 = H1 * (n_meas / 40)
        prior = {"kind": "gaussian", "mean": mu, "cov": Gam}
        pts, w = _sigma_points(mu, Gam)
        vals = [laplace.dkl_hat(H1, p, prior)[0] for p in pts]
        I4 = laplace.eig_average(vals, w)
        ref4 = 0.5 * np.linalg.slogdet(Gam @ H1)[1]
        assert abs(I4 - ref4) < 1e-11 * abs(ref4)
        exact = 0.5 * np.linalg.slogdet(np.eye(N) + Gam @ H1)[1]
        gaps.append(exact - I4)
    assert all(g > 0 for g in gaps)
    assert 9.0 < gaps[0] / gaps[1] < 11.0 and 9.0 < gaps[1] / gaps[2] < 11.0
    del rng


def test_design_eval_and_greedy():
    rng = np.random.default_rng(4)
    S, C = 5, 8
    lo = np.zeros(N)
    hi = np.ones(N)
    prior = laplace.uniform_prior(lo, hi)
    H1r = np.empty((S, C, N, N))
    for s in range(S):
        for c in range(C):
            G = rng.standard_normal((9, N))
            H1r[s, c] = G.T @ G * 50
    theta = rng.uniform(0, 1, (S, N))
    w = np.full(S, 1.0 / S)
    order, curve = laplace.greedy(H1r, theta, w, prior, 5)
    assert np.all(np.diff(curve) > 0)           # adding PSD terms raises log det
    chosen = []
    for k in range(len(order)):
        masks = []
        cands = [c for c in range(C) if c not in chosen]
        for c in cands:
            m = np.zeros(C, np.uint8)
            m[chosen + [c]] = 1
            masks.append(m)
        vals = laplace.design_eval(H1r, np.array(masks), theta, w, prior)
        finite = np.where(np.isnan(vals), -np.inf, vals)
        assert cands[int(np.argmax(finite))] == order[k]
        assert abs(np.max(finite) - curve[k]) < 1e-12 * abs(curve[k])
        chosen.append(int(order[k]))
    # first step of greedy on tiny sets: brute force over all pairs bounds it
    best_pair = max(laplace.design_eval(H1r, np.array([np.isin(np.arange(C), p).astype(np.uint8)
                                                       for p in itertools.combinations(range(C), 2)]),
                                        theta, w, prior))
    assert curve[1] <= best_pair + 1e-12


def test_stacked_dkl_and_greedy_step_values_equal_the_scalar_forms():
    # the stacked Theorem 4 formula against dkl_hat one matrix at a time,
    # including a Hessian with a zero diagonal and an indefinite one (NaN),
    # and the per-candidate step values against design_eval's sums
    rng = np.random.default_rng(12)
    S, C = 6, 9
    lo, hi = -np.ones(N), 2 * np.ones(N)
    prior = laplace.uniform_prior(lo, hi)
    H1r = np.empty((S, C, N, N))
    for s in range(S):
        for c in range(C):
            H1r[s, c] = _spd(rng, np.logspace(-3, 5, N)[rng.permutation(N)])
    H1r[2, 4] = 0.0
    H1r[4, 7] = -np.eye(N) + 0.1 * np.ones((N, N))
    theta = rng.uniform(-1, 2, (S, N))
    got = laplace.dkl_hat_stack(H1r, np.repeat(theta[:, None], C, axis=1), prior)
    for s in range(S):
        for c in range(C):
            ref, ok = laplace.dkl_hat(H1r[s, c], theta[s], prior)
            if ok:
                assert abs(got[s, c] - ref) <= 1e-12 * abs(ref)
            else:
                assert np.isnan(got[s, c]) and (s, c) in ((2, 4), (4, 7))
    w = rng.uniform(-0.5, 1.5, S)
    base = H1r[:, 1] + H1r[:, 3]
    vals = laplace.greedy_step_values(H1r, base, theta, w, prior)
    masks = np.zeros((C, C), np.uint8)
    masks[:, [1, 3]] = 1
    masks[np.arange(C), np.arange(C)] = 1
    ref = laplace.design_eval(H1r, masks, theta, w, prior)
    rest = np.array([c for c in range(C) if c not in (1, 3)])   # not yet chosen
    vals, ref = vals[rest], ref[rest]
    fin = ~np.isnan(ref)
    assert np.array_equal(fin, ~np.isnan(vals)) and not fin.all()
    assert np.max(np.abs(vals[fin] - ref[fin])) <= 1e-12 * np.max(np.abs(ref[fin]))


def _golden_sizes():
    path = os.path.join(os.path.dirname(__file__), "golden", "sparse_grid_sizes.txt")
    rows = []
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(tuple(int(v) for v in line.split()))
    return rows


@pytest.mark.parametrize("d,w,count", [r for r in _golden_sizes() if r[2] < 20000])
def test_sparse_grid_sizes_match_paper(d, w, count):
    X, W = smolyak.sparse_grid(d, w)
    assert len(W) == count
    assert abs(W.sum() - 1.0) < 1e-12


@pytest.mark.slow
@pytest.mark.parametrize("d,w,count", [r for r in _golden_sizes() if r[2] >= 20000])
def test_sparse_grid_sizes_match_paper_large(d, w, count):
    X, W = smolyak.sparse_grid(d, w)
    assert len(W) == count


@pytest.mark.parametrize("d,w", [(2, 4), (3, 3), (7, 3)])
def test_sparse_grid_exact_on_total_degree(d, w):
    X, W = smolyak.sparse_grid(d, w)
    rng = np.random.default_rng(5)
    for _ in range(25):
        deg = rng.integers(0, 2 * w + 2)
        p = np.zeros(d, int)
        for _ in range(deg):
            p[rng.integers(d)] += 1
        approx = np.sum(W * np.prod(X**p, axis=1))
        exact = np.prod([(1.0 / (q + 1)) if q % 2 == 0 else 0.0 for q in p])
        assert abs(approx - exact) < 1e-12, (p, approx, exact)
    # one degree higher is not integrated exactly for every monomial
    p = np.zeros(d, int)
    p[0] = 2 * w + 2
    assert abs(np.sum(W * X[:, 0] ** p[0]) - 1.0 / (2 * w + 3)) > 1e-10


def test_sparse_grid_box_mapping():
    lo = np.array([1.0, -2.0, 10.0])
    hi = np.array([3.0, 2.0, 11.0])
    X, W = smolyak.sparse_grid(3, 4, lo, hi)
    assert np.all(X >= lo) and np.all(X <= hi)
    assert np.allclose(np.sum(W[:, None] * X, axis=0), 0.5 * (lo + hi), rtol=0, atol=1e-12)
