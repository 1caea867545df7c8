"""Comparison helpers shared by the GPU parity tests (any method arithmetic
they need comes from the oracle).

Receiver traces and Jacobian columns are compared per receiver as well as
as a whole, so that one bad receiver cannot hide under the norm of the
others: for arrays laid out [levels][receivers][...], every receiver whose
reference norm is at least `floor` (1 %) of the largest receiver's must
match to relative L2 `tol` on its own; the rest must match to `tol` times
the largest receiver's norm.  Below the floor sit receivers the wave only
begins to reach within the record (or next to a rigid edge, where the
field is pinned near zero): their few small values carry the FP32 rounding
of the much larger field that produced them (measured: 2.4e-5 relative at
a receiver holding 0.1 % of the strongest one's norm, whose error is
2.6e-8 of the strongest norm).
"""
import numpy as np


def receiver_relerr(a, b):
    """Per-receiver relative L2 errors of a against b ([nt][nrec][...]) and
    the per-receiver reference norms."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    axes = tuple(k for k in range(b.ndim) if k != 1)
    nb = np.sqrt(np.sum(b * b, axis=axes))
    nd = np.sqrt(np.sum((a - b) ** 2, axis=axes))
    return nd / np.maximum(nb, 1e-300), nd, nb


def check_receivers(a, b, tol, floor=1e-2, what=""):
    """Asserts the whole-array and per-receiver bounds described above and
    returns the largest relative error over the receivers held to it."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    whole = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    assert whole <= tol, (what, "whole", whole)
    rel, nd, nb = receiver_relerr(a, b)
    top = float(nb.max())
    if top == 0.0:
        assert float(nd.max()) == 0.0, (what, "reference is zero")
        return 0.0
    strong = nb >= floor * top
    worst = int(np.argmax(np.where(strong, rel, -1.0)))
    assert rel[strong].max() <= tol, (what, "receiver", worst, float(rel[worst]))
    assert float(nd[~strong].max(initial=0.0)) <= tol * top, (what, "weak receivers")
    return float(rel[strong].max())


def check_jacobian(Jg, Jr, tol, floor=1e-2, what=""):
    """check_receivers on every Jacobian column ([nt][nrec][2][7]); returns
    the largest per-receiver relative error over the columns."""
    return max(check_receivers(Jg[..., j], Jr[..., j], tol, floor, f"{what} column {j}")
               for j in range(Jr.shape[-1]))


def logdet_rounding(Hs, w):
    """Bound on the FP64 rounding of sum_s w_s (1/2) log det Hs[s] taken by a
    backward-stable Cholesky of the diagonally scaled Hessian:
    sum_s |w_s| n^2 eps kappa(H~_s) (two different operation orders, such as
    the device's and LAPACK's, may differ by up to twice this)."""
    n = Hs.shape[-1]
    d = np.sqrt(np.abs(np.diagonal(Hs, axis1=-2, axis2=-1)))
    Ht = Hs / (d[..., :, None] * d[..., None, :])
    kappa = np.linalg.cond(Ht)
    return float(np.sum(np.abs(w) * n * n * np.finfo(np.float64).eps * kappa))


def check_greedy(order, curve, H1r, theta, w, prior, rel_tie=1e-9, ref_H1r=None,
                 ref_gap=None):
    """Holds a greedy run (order, curve) to the oracle's design sums, step
    by step on the run's own prefix of chosen receivers:
      - with the same per-candidate Hessians H1r, the pick is an argmax of
        I(prefix + {c}) over the candidates not chosen yet and the reported
        value is that I, both within rel_tie * |I| plus twice the log-det
        rounding bound of the designs compared (logdet_rounding: only badly
        conditioned designs, such as single receivers, widen it);
      - with ref_H1r (the oracle's own Hessians, which differ by rounding of
        the solves), the pick must also be the oracle's argmax wherever the
        oracle's two best candidates are more than ref_gap apart.
    Uses the oracle (oracle.laplace.greedy_step_values)."""
    from oracle import laplace
    S, C = H1r.shape[:2]
    base = np.zeros((S, 7, 7))
    base_ref = np.zeros((S, 7, 7))
    chosen = []
    for k, c in enumerate(np.asarray(order).tolist()):
        vals = laplace.greedy_step_values(H1r, base, theta, w, prior)
        vals[chosen] = np.nan
        if c < 0:
            assert np.isnan(vals).all(), (k, "stopped with candidates left")
            assert np.isnan(curve[k])
            continue
        assert c not in chosen, (k, c)
        best = np.nanmax(vals)
        cb = int(np.nanargmax(vals))
        r_c = logdet_rounding(base + H1r[:, c], w)
        r_b = logdet_rounding(base + H1r[:, cb], w)
        tol = rel_tie * max(1.0, abs(best)) + 2 * (r_c + r_b)
        assert vals[c] >= best - tol, (k, c, float(vals[c]), float(best), tol)
        tol_v = rel_tie * max(1.0, abs(vals[c])) + 2 * r_c
        assert abs(curve[k] - vals[c]) <= tol_v, (k, float(curve[k]), float(vals[c]), tol_v)
        if ref_H1r is not None:
            rv = laplace.greedy_step_values(ref_H1r, base_ref, theta, w, prior)
            rv[chosen] = np.nan
            top2 = np.sort(rv[~np.isnan(rv)])[-2:]
            if len(top2) == 2 and top2[1] - top2[0] > ref_gap:
                assert c == int(np.nanargmax(rv)), (k, c, int(np.nanargmax(rv)))
            base_ref = base_ref + ref_H1r[:, c]
        chosen.append(c)
        base = base + H1r[:, c]
    return chosen


def scaled_hessian_err(Hg, Hr):
    """max |Hg - Hr|_ij / sqrt(Hr_ii Hr_jj) over the last two axes.  For
    H = J^T J and Jacobian columns within relative eps, Cauchy-Schwarz bounds
    this by 2 eps + eps^2."""
    Hg = np.asarray(Hg, dtype=np.float64)
    Hr = np.asarray(Hr, dtype=np.float64)
    d = np.sqrt(np.abs(np.diagonal(Hr, axis1=-2, axis2=-1)))
    sc = d[..., :, None] * d[..., None, :]
    return float(np.max(np.abs(Hg - Hr) / np.maximum(sc, 1e-300)))
