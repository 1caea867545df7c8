"""Writes the oracle's expected values for the two full-size parity cases.

Each case is one prior sample at a configuration whose oracle solves take
minutes (15 leapfrog solves of 8.4e9 or 4.2e9 grid-point updates each), too
long to rerun inside a GPU test.  This script calls only the FP64 oracle
(`oracle/`) and the seeded input generator (`synthetic/`); nothing here
touches the HIP library.  Usage (from the repository root):

    python tests/golden/make_fullsize_golden.py [c5|c4|all] [--threads N]

Outputs (numpy .npz, no pickled objects):
  c5_node_fullsize.npz   2048 x 1024 grid, 4000 steps, nodal 6-layer medium
                         with the 5 % random-field perturbation, the centre
                         node of the level-3 sparse grid (every parameter at
                         its prior mean), noise level from the nominal solve
                         at the prior mean (1e-3 x peak), 201 candidate
                         receivers: H_1 per candidate (Theorem 2, additive
                         over receivers), their sum, D^_KL of the whole
                         array (Theorem 4), nominal traces at 9 candidates
                         and Jacobian columns at 5 of them.
  c4_sample_fullsize.npz 1024^2 grid, 4000 steps, random 4-layer medium,
                         101 random receivers, sample 1 of the 64-sample
                         query (the first whose P wave reaches the surface
                         halfway through the record), sigma = 0.5 given:
                         H_1 per receiver and in total, D^_KL, nominal
                         traces at 5 receivers, Jacobian columns at 3.

Nominal traces and H_1 are stored in FP64.  The sampled Jacobian columns are
stored rounded to FP32 (relative rounding 6e-8, far below the 1e-3 Jacobian
tolerance) to keep the files small.  Each file also holds SHA-256 digests of
its inputs, so that a test can tell a changed input from a parity failure.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synthetic  # noqa: E402
from oracle import elastic, laplace, smolyak  # noqa: E402

C5_FILE = os.path.join(HERE, "c5_node_fullsize.npz")
C4_FILE = os.path.join(HERE, "c4_sample_fullsize.npz")
C4_SAMPLE = 1
C4_SIGMA = 0.5
C5_TRACE_CANDS = np.arange(0, 201, 25)
C5_JAC_CANDS = np.arange(0, 201, 50)
C4_TRACE_RECS = np.arange(0, 101, 25)
C4_JAC_RECS = np.arange(0, 101, 50)


def input_digest(*arrays) -> str:
    """SHA-256 over the raw bytes of the given arrays (FP64 / int32)."""
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def medium_digest(wl) -> str:
    g = wl.grid
    return input_digest(wl.medium.rho, wl.medium.lam, wl.medium.mu,
                        np.array([g.nx, g.nz, g.nsteps]), np.array([g.h, g.dt]),
                        np.asarray(wl.receivers, dtype=np.int32))


def c5_centre_node(wl):
    """The level-3 sparse-grid node at the centre of the prior box."""
    X, _ = smolyak.sparse_grid(7, 3, wl.lo, wl.hi)
    mid = 0.5 * (wl.lo + wl.hi)
    k = int(np.argmin(np.max(np.abs(X - mid) / (wl.hi - wl.lo), axis=1)))
    assert np.allclose(X[k], mid, rtol=1e-14, atol=0)
    return X[k]


def _sample(wl, theta, sigma, pool, extra=None):
    """Literal 15-solve Jacobian of one sample on the pool's threads (plus
    any extra jobs submitted alongside, e.g. the noise solve)."""
    fut = pool.submit(lambda: None) if extra is None else pool.submit(extra)
    nominal, J = elastic.jacobian_literal(wl.grid, wl.medium, theta, wl.receivers,
                                          wl.rel_step, wl.stf, pool=pool)
    return nominal, J, fut.result()


def make_c5(threads):
    wl = synthetic.config("c5")[0]
    theta = c5_centre_node(wl)
    t0 = time.time()
    with ThreadPoolExecutor(threads) as pool:
        # the noise level needs the nominal solve at the prior mean, which is
        # this node; it is run once more over all surface nodes
        nominal, J, sigma = _sample(
            wl, theta, None, pool,
            extra=lambda: elastic.noise_sigma(wl.grid, wl.medium, wl.theta_bar,
                                              wl.noise_rel, wl.stf))
    H1r = laplace.hessian_h1_per_receiver(J, sigma)
    H1 = H1r.sum(axis=0)
    prior = laplace.uniform_prior(wl.lo, wl.hi)
    dkl, ok = laplace.dkl_hat(H1, theta, prior)
    assert ok, "c5 centre node: H_1 not positive definite"
    np.savez_compressed(
        C5_FILE, theta=theta, sigma=np.float64(sigma), H1r=H1r, H1=H1,
        dkl=np.float64(dkl), trace_cands=C5_TRACE_CANDS,
        nominal=nominal[:, C5_TRACE_CANDS], jac_cands=C5_JAC_CANDS,
        J=J[:, C5_JAC_CANDS].astype(np.float32),
        input_sha256=np.array(medium_digest(wl)), rel_step=np.float64(wl.rel_step),
        seconds=np.float64(time.time() - t0))
    print(f"c5: sigma={sigma:.6e} dkl={dkl:.9f} in {time.time() - t0:.0f} s", flush=True)


def make_c4(threads):
    wl = synthetic.c4_largest_query()
    theta = wl.theta[C4_SAMPLE]
    t0 = time.time()
    with ThreadPoolExecutor(threads) as pool:
        nominal, J, _ = _sample(wl, theta, C4_SIGMA, pool)
    H1r = laplace.hessian_h1_per_receiver(J, C4_SIGMA)
    H1 = H1r.sum(axis=0)
    prior = laplace.uniform_prior(wl.lo, wl.hi)
    dkl, ok = laplace.dkl_hat(H1, theta, prior)
    assert ok, "c4 sample: H_1 not positive definite"
    np.savez_compressed(
        C4_FILE, sample=np.int64(C4_SAMPLE), theta=theta, sigma=np.float64(C4_SIGMA),
        H1r=H1r, H1=H1, dkl=np.float64(dkl), trace_recs=C4_TRACE_RECS,
        nominal=nominal[:, C4_TRACE_RECS], jac_recs=C4_JAC_RECS,
        J=J[:, C4_JAC_RECS].astype(np.float32),
        input_sha256=np.array(medium_digest(wl)), rel_step=np.float64(wl.rel_step),
        seconds=np.float64(time.time() - t0))
    print(f"c4: dkl={dkl:.9f} in {time.time() - t0:.0f} s", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="?", default="all", choices=["c5", "c4", "all"])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    if a.which in ("c4", "all"):
        make_c4(a.threads)
    if a.which in ("c5", "all"):
        make_c5(a.threads)


if __name__ == "__main__":
    main()
