"""Oracle sparse quadrature (Section 3.3.4, "Numerical integration"):
Smolyak combination of 1-D Gauss-Legendre rules over a total-degree index set.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Reading of the paper: the 1-D rule of level i has m(i) = i Gauss-Legendre
points, the index set is {i >= 1 : sum_n (i_n - 1) <= w} (Section 4.3 names
Gauss-Legendre sparse grids on total-degree index sets), and the combination
technique gives
    Q_w = sum_{w-d+1 <= |i-1| <= w} (-1)^{w-|i-1|} C(d-1, w-|i-1|) (x)_n Q_{i_n},
with coincident nodes merged (weights added).  Weights integrate against the
uniform density on the box, so they sum to one.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def gauss_legendre_unit(m: int):
    """m-point Gauss-Legendre rule on [-1, 1] for the density 1/2."""
    x, w = np.polynomial.legendre.leggauss(m)
    return x, 0.5 * w


def index_set(d: int, w: int):
    """All i in N^d, i_n >= 1, with sum(i_n - 1) <= w."""
    out = []
    for t in itertools.product(range(w + 1), repeat=d):
        if sum(t) <= w:
            out.append(tuple(v + 1 for v in t))
    return out


def sparse_grid(d: int, w: int, lo=None, hi=None, merge_tol: float = 1e-12):
    """Nodes [eta][d] and weights [eta] of the level-w rule on the box
    [lo, hi] (default [-1, 1]^d)."""
    acc = {}
    for idx in index_set(d, w):
        q = sum(i - 1 for i in idx)
        if q < w - d + 1:
            continue
        coef = (-1) ** (w - q) * math.comb(d - 1, w - q)
        rules = [gauss_legendre_unit(i) for i in idx]
        for pick in itertools.product(*[range(len(r[0])) for r in rules]):
            x = tuple(rules[n][0][p] for n, p in enumerate(pick))
            wt = coef * math.prod(rules[n][1][p] for n, p in enumerate(pick))
            key = tuple(int(round(v / merge_tol)) for v in x)
            if key in acc:
                acc[key][1] += wt
            else:
                acc[key] = [np.array(x), wt]
    keys = sorted(acc)
    X = np.array([acc[k][0] for k in keys]).reshape(len(keys), d)
    W = np.array([acc[k][1] for k in keys])
    if lo is not None:
        lo = np.asarray(lo, dtype=np.float64)
        hi = np.asarray(hi, dtype=np.float64)
        X = lo + 0.5 * (X + 1.0) * (hi - lo)
    return X, W
