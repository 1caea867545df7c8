"""Oracle Laplace-EIG arithmetic: Gauss-Newton Hessian, scaled log-det,
KL divergence estimate, quadrature averages, design sums and greedy search.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain FP64 numpy.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

NTHETA = 7


def hessian_h1(J: np.ndarray, sigma: float) -> np.ndarray:
    """H_1 = sum_{r,m} grad g_r^T C_eps^-1 grad g_r with C_eps = sigma^2 I
    (Theorem 2, eq. for H_1; Section 3.3.2, eq. for H_I with the receiver
    selection Hessian diag(1/sigma^2)).  J has shape [..., 7]."""
    Jf = J.reshape(-1, J.shape[-1])
    return (Jf.T @ Jf) / (sigma * sigma)


def hessian_h1_per_receiver(J: np.ndarray, sigma: float) -> np.ndarray:
    """One H_1 per receiver r (J shape [nt][nrec][2][7]); their sum over r is
    H_1 (the double sum over receivers and times is additive)."""
    out = np.empty((J.shape[1], J.shape[-1], J.shape[-1]))
    for r in range(J.shape[1]):
        out[r] = hessian_h1(J[:, r], sigma)
    return out


def logdet_scaled(H: np.ndarray):
    """log det H via the scaled Hessian of Section 3.3.3:
    S = sqrt(diag H), H~ = S^-T H S^-1, log det H = log det H~ + 2 sum log S.
    Returns (logdet, ok); ok is False when H~ is not positive definite."""
    d = np.diag(H)
    if not np.all(np.isfinite(H)) or np.any(d <= 0):
        return float("nan"), False
    s = np.sqrt(d)
    Ht = H / np.outer(s, s)
    try:
        L = np.linalg.cholesky(Ht)
    except np.linalg.LinAlgError:
        return float("nan"), False
    return float(2.0 * np.sum(np.log(np.diag(L))) + 2.0 * np.sum(np.log(s))), True


def log_prior(theta, prior: dict) -> float:
    """h(theta) = log p(theta) (Section 2.2, after the cost functional)."""
    theta = np.asarray(theta, dtype=np.float64)
    if prior["kind"] == "uniform":
        lo, hi = np.asarray(prior["lo"]), np.asarray(prior["hi"])
        return -float(np.sum(np.log(hi - lo)))
    if prior["kind"] == "gaussian":
        mean, cov = np.asarray(prior["mean"]), np.asarray(prior["cov"])
        r = theta - mean
        n = r.size
        sign, ld = np.linalg.slogdet(cov)
        return float(-0.5 * r @ np.linalg.solve(cov, r)
                     - 0.5 * (n * math.log(2 * math.pi) + ld))
    raise ValueError(prior["kind"])


def dkl_hat(H1: np.ndarray, theta, prior: dict):
    """Theorem 4:  D^_KL = -1/2 log((2 pi)^N |H_1^-1|) - N/2 - h(theta).
    Returns (value, ok)."""
    n = H1.shape[0]
    ld, ok = logdet_scaled(H1)
    if not ok:
        return float("nan"), False
    return (-0.5 * (n * math.log(2 * math.pi) - ld) - 0.5 * n
            - log_prior(theta, prior)), True


def dkl_hat_stack(H1: np.ndarray, theta: np.ndarray, prior: dict) -> np.ndarray:
    """dkl_hat over a stack of Hessians H1 [..., N, N] with theta [..., 7]
    (the same Theorem 4 formula and scaled log-det of Section 3.3.3, with
    numpy's stacked Cholesky); NaN where a Hessian is not positive definite.
    Only for the uniform prior, whose h does not depend on theta."""
    if prior["kind"] != "uniform":
        raise ValueError("dkl_hat_stack: uniform prior only")
    n = H1.shape[-1]
    d = np.diagonal(H1, axis1=-2, axis2=-1)
    ok = np.all(np.isfinite(H1), axis=(-2, -1)) & np.all(d > 0, axis=-1)
    s = np.sqrt(np.where(ok[..., None], d, 1.0))
    Ht = H1 / (s[..., :, None] * s[..., None, :])
    Ht = np.where(ok[..., None, None], Ht, np.eye(n))
    ld = np.full(H1.shape[:-2], np.nan)
    flat_H = Ht.reshape(-1, n, n)
    flat_ok = ok.reshape(-1)
    flat_ld = ld.reshape(-1)
    try:
        L = np.linalg.cholesky(flat_H)
        good = flat_ok
    except np.linalg.LinAlgError:
        # some scaled Hessian is indefinite: factor one by one
        L = np.zeros_like(flat_H)
        good = flat_ok.copy()
        for q in range(flat_H.shape[0]):
            try:
                L[q] = np.linalg.cholesky(flat_H[q])
            except np.linalg.LinAlgError:
                good[q] = False
    diagL = np.diagonal(L, axis1=-2, axis2=-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        v = 2.0 * np.sum(np.log(diagL), axis=-1) + \
            2.0 * np.sum(np.log(s.reshape(-1, n)), axis=-1)
    flat_ld[good] = v[good]
    h = log_prior(np.zeros(7), prior)
    return -0.5 * (n * math.log(2 * math.pi) - ld) - 0.5 * n - h


def greedy_step_values(H1r: np.ndarray, base: np.ndarray, theta: np.ndarray,
                       w: np.ndarray, prior: dict) -> np.ndarray:
    """I(design + {c}) = sum_s w_s D^_KL(base_s + H_1,c(s)) for every
    candidate c, where base holds the chosen receivers' summed Hessians
    [S][7][7] (H_1 additive over receivers, Section 4.5 designs)."""
    vals = dkl_hat_stack(base[:, None] + H1r, theta[:, None], prior)   # [S][C]
    return np.sum(np.asarray(w)[:, None] * vals, axis=0)


def eig_average(dkl: np.ndarray, w: np.ndarray) -> float:
    """I = sum_i w_i D^_KL(theta_i) (eqs. for the sparse-quadrature and Monte
    Carlo estimates).  Any failed sample (NaN) makes I NaN."""
    return float(np.sum(np.asarray(w) * np.asarray(dkl)))


def uniform_prior(lo, hi) -> dict:
    return {"kind": "uniform", "lo": np.asarray(lo, dtype=np.float64),
            "hi": np.asarray(hi, dtype=np.float64)}


def design_eval(H1r: np.ndarray, masks: np.ndarray, theta: np.ndarray,
                w: np.ndarray, prior: dict) -> np.ndarray:
    """EIG of each design: I(xi) = sum_s w_s D^_KL(sum_{r in xi} H_1,r(s)).
    H1r [S][C][7][7], masks [D][C] (0/1)."""
    S = H1r.shape[0]
    out = np.empty(masks.shape[0])
    for d in range(masks.shape[0]):
        sel = np.nonzero(masks[d])[0]
        vals = np.empty(S)
        for s in range(S):
            vals[s], _ = dkl_hat(H1r[s, sel].sum(axis=0), theta[s], prior)
        out[d] = eig_average(vals, w)
    return out


def greedy(H1r: np.ndarray, theta: np.ndarray, w: np.ndarray, prior: dict,
           kmax: int):
    """Greedy receiver selection: repeatedly add the candidate that maximises
    I(xi + {c}); ties go to the lowest index; a candidate whose I is NaN is
    never preferred.  Returns (order, curve)."""
    S, C = H1r.shape[:2]
    chosen = []
    curve = []
    base = np.zeros((S, NTHETA, NTHETA))
    for _ in range(min(kmax, C)):
        best, best_c = -np.inf, -1
        for c in range(C):
            if c in chosen:
                continue
            vals = np.array([dkl_hat(base[s] + H1r[s, c], theta[s], prior)[0]
                             for s in range(S)])
            val = eig_average(vals, w)
            if np.isnan(val):
                continue
            if val > best:
                best, best_c = val, c
        if best_c < 0:
            break
        chosen.append(best_c)
        curve.append(best)
        base = base + H1r[:, best_c]
    return np.array(chosen, dtype=np.int64), np.array(curve)
