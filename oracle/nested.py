"""Oracle nested (double-loop) Monte Carlo estimate of the expected
information gain (TEST INFRASTRUCTURE ONLY).

The expected information gain is the prior-and-data average of the log
ratio of posterior to prior, which for a likelihood p(y | theta) equals
E[log p(y | theta*) - log p(y)] with p(y) the evidence (eq. for I, Section
2.2).  The direct sample-average estimator draws outer pairs (theta*_n,
y_n = g(theta*_n) + eps_n) and replaces p(y_n) by an inner average over
prior draws theta_m (the double-loop estimator of the introduction and of
Section 4.4, where the inner samples reuse the outer ones).  With
C_eps = sigma^2 I the Gaussian normalisers cancel:

    log-ratio_n = -|eps_n|^2 / (2 sigma^2)
                  - log( (1/M) sum_m exp(-|y_n - g(theta_m)|^2 / (2 sigma^2)) ).

Plain FP64 numpy, one outer sample at a time.
"""
from __future__ import annotations

import numpy as np


def log_ratios(g_outer: np.ndarray, noise: np.ndarray, g_inner: np.ndarray,
               sigma: float) -> np.ndarray:
    """g_outer [N][K] model outputs at theta*_n, noise [N][K] standard normal
    draws (eps_n = sigma * noise_n), g_inner [M][K] outputs at the inner
    prior draws.  Returns the N log ratios."""
    g_outer = np.asarray(g_outer, dtype=np.float64)
    g_inner = np.asarray(g_inner, dtype=np.float64)
    noise = np.asarray(noise, dtype=np.float64)
    M = g_inner.shape[0]
    out = np.empty(g_outer.shape[0])
    for n in range(g_outer.shape[0]):
        y = g_outer[n] + sigma * noise[n]
        ll = -np.sum((y[None, :] - g_inner) ** 2, axis=1) / (2.0 * sigma * sigma)
        top = ll.max()
        log_evidence = top + np.log(np.sum(np.exp(ll - top))) - np.log(M)
        out[n] = -0.5 * np.sum(noise[n] ** 2) - log_evidence
    return out


def eig_nested(g_outer, noise, g_inner, sigma) -> float:
    """Mean of the log ratios over the outer samples."""
    return float(np.mean(log_ratios(g_outer, noise, g_inner, sigma)))
