"""Pins of the oracle's nested Monte Carlo EIG (CPU only).

For a linear model g(theta) = A theta with a Gaussian prior N(0, Gamma) and
C_eps = sigma^2 I the expected information gain has the closed form
1/2 log det(I + sigma^-2 Gamma A^T A); the double-loop estimator must
converge to it (its bias is O(1/M), positive), and the Laplace form of
Theorem 4 averaged over the prior gives 1/2 log det(Gamma H_1) which it
exceeds by 1/2 log det(I + (Gamma H_1)^-1).
"""
import math

import numpy as np

from oracle import laplace, nested


def _linear_case(rng, d=2, K=12, scale=0.6):
    A = rng.standard_normal((K, d)) * scale
    Gamma = np.diag(rng.uniform(0.5, 1.5, d))
    sigma = 0.7
    exact = 0.5 * np.linalg.slogdet(np.eye(d) + Gamma @ A.T @ A / sigma**2)[1]
    return A, Gamma, sigma, exact


def test_nested_mc_converges_to_closed_form():
    rng = np.random.default_rng(0)
    A, Gamma, sigma, exact = _linear_case(rng)
    N = 3000
    th_out = rng.multivariate_normal(np.zeros(2), Gamma, N)
    th_in = rng.multivariate_normal(np.zeros(2), Gamma, 6000)
    noise = rng.standard_normal((N, A.shape[0]))
    lr = nested.log_ratios(th_out @ A.T, noise, th_in @ A.T, sigma)
    est, se = lr.mean(), lr.std(ddof=1) / math.sqrt(N)
    assert abs(est - exact) < 4 * se + 0.01, (est, exact, se)


def test_nested_mc_bias_shrinks_with_inner_count():
    # the evidence estimate is unbiased but its log is biased low, so the
    # estimator is biased high, by less as M grows (common random numbers)
    rng = np.random.default_rng(1)
    A, Gamma, sigma, exact = _linear_case(rng, d=2, K=20, scale=1.0)
    N = 2000
    th_out = rng.multivariate_normal(np.zeros(2), Gamma, N)
    noise = rng.standard_normal((N, A.shape[0]))
    th_in = rng.multivariate_normal(np.zeros(2), Gamma, 8000)
    ests = [nested.eig_nested(th_out @ A.T, noise, th_in[:M] @ A.T, sigma)
            for M in (50, 400, 8000)]
    assert ests[0] > ests[1] > ests[2] > exact - 0.05, (ests, exact)


def test_laplace_gap_on_linear_model():
    # Theorem 4 on the linear-Gaussian model: H_1 = A^T A / sigma^2 at every
    # theta; the prior average of D^_KL is 1/2 log det(Gamma H_1) (up to the
    # prior term's mean), the exact EIG exceeds it by 1/2 log det(I + (Gamma H_1)^-1)
    rng = np.random.default_rng(2)
    A, Gamma, sigma, exact = _linear_case(rng, d=2, K=40, scale=2.0)
    H1 = A.T @ A / sigma**2
    prior = {"kind": "gaussian", "mean": np.zeros(2), "cov": Gamma}
    ths = rng.multivariate_normal(np.zeros(2), Gamma, 20000)
    lap = np.mean([laplace.dkl_hat(H1, th, prior)[0] for th in ths])
    want = 0.5 * np.linalg.slogdet(Gamma @ H1)[1]
    assert abs(lap - want) < 0.03
    gap = 0.5 * np.linalg.slogdet(np.eye(2) + np.linalg.inv(Gamma @ H1))[1]
    assert abs(exact - want - gap) < 1e-10


def test_reused_inner_samples_include_the_true_parameter():
    # with the inner set equal to the outer set, the n-th inner term is the
    # outer sample's own likelihood: each log ratio is <= log M
    rng = np.random.default_rng(3)
    A, Gamma, sigma, _ = _linear_case(rng)
    th = rng.multivariate_normal(np.zeros(2), Gamma, 300)
    noise = rng.standard_normal((300, A.shape[0]))
    g = th @ A.T
    lr = nested.log_ratios(g, noise, g, sigma)
    assert np.all(lr <= math.log(300) + 1e-12)
    # and M = 1 with reuse gives exactly zero
    assert abs(nested.log_ratios(g[:1], noise[:1], g[:1], sigma)[0]) < 1e-12
