"""Oracle composition of one design query (TEST INFRASTRUCTURE ONLY).

Per prior sample: 1 nominal + 2*7 perturbed solves -> central-difference
Jacobian (or 1 + 7 forward-sensitivity solves, Algorithm 1) -> H_1 -> D^_KL; then the weighted average over samples
(Theorem 4 with the Monte Carlo or sparse-quadrature rule of Section 3.3.4).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from typing import Optional

import numpy as np

from . import elastic, laplace


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def sample_terms(wl, theta, sigma, per_receiver=False, jacobian="fd", pool=None):
    if jacobian == "fd":
        nominal, J = elastic.jacobian_literal(wl.grid, wl.medium, theta, wl.receivers,
                                              wl.rel_step, wl.stf, pool=pool)
    elif jacobian == "sensitivity":
        nominal, J = elastic.jacobian_sensitivity(wl.grid, wl.medium, theta, wl.receivers,
                                                  wl.stf)
    else:
        raise ValueError(jacobian)
    if per_receiver:
        H = laplace.hessian_h1_per_receiver(J, sigma)
    else:
        H = laplace.hessian_h1(J, sigma)
    return nominal, J, H


def query(wl, theta=None, weights=None, sigma: Optional[float] = None,
          per_receiver=False, threads: Optional[int] = None, keep_J=False,
          jacobian="fd"):
    """Runs the whole path for one workload query.  Returns a dict with sigma,
    nominal traces, (J), H1 [S][7][7] (or [S][R][7][7]), dkl [S], eig."""
    theta = wl.theta if theta is None else np.asarray(theta)
    weights = wl.weights if weights is None else np.asarray(weights)
    if sigma is None and getattr(wl, "sigma", None) is not None:
        sigma = wl.sigma
    if sigma is None:
        sigma = elastic.noise_sigma(wl.grid, wl.medium, wl.theta_bar,
                                    wl.noise_rel, wl.stf)
    prior = laplace.uniform_prior(wl.lo, wl.hi)
    nthr = threads or default_threads()
    if len(theta) < nthr and jacobian == "fd":
        # few samples: spread each sample's 15 solves over the threads instead
        # (each solve stays single-threaded; the C solver releases the GIL)
        with ThreadPoolExecutor(nthr) as pool:
            res = [sample_terms(wl, th, sigma, per_receiver, jacobian, pool) for th in theta]
    else:
        with ThreadPoolExecutor(nthr) as pool:
            res = list(pool.map(lambda th: sample_terms(wl, th, sigma, per_receiver, jacobian),
                                list(theta)))
    H = np.stack([r[2] for r in res])
    Htot = H.sum(axis=1) if per_receiver else H
    dkl = np.array([laplace.dkl_hat(Htot[s], theta[s], prior)[0]
                    for s in range(len(theta))])
    out = {"sigma": sigma, "nominal": np.stack([r[0] for r in res]), "H1": H,
           "dkl": dkl, "eig": laplace.eig_average(dkl, weights)}
    if keep_J:
        out["J"] = np.stack([r[1] for r in res])
    return out
