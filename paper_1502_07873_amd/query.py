"""One design query through the C ABI (marshalling only).

sigma (noise_sigma_peak at the prior mean) -> jacobian_fd (1 + 2*7 solves per
sample, J, H_1) or jacobian_sensitivity (1 + 7 solves) -> laplace_eig (scaled log-det, D^_KL, weighted average), or
design_eval / design_greedy on per-receiver Hessians.
"""
from __future__ import annotations

import numpy as np
import torch

from . import eigseis


def device_medium(kind: str, rho, lam, mu, device="cuda"):
    k = eigseis.MEDIUM_NODAL if kind == "nodal" else eigseis.MEDIUM_LAYERED
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64),  # noqa: E731
                                  device=device)
    return (k, t(rho), t(lam), t(mu))


def grid_tuple(g):
    return (g.nx, g.nz, g.h, g.dt, g.nsteps, eigseis.BC_CODES[getattr(g, "bc", "rigid")])


def run_query(ctx: eigseis.Context, grid, medium, receivers, lo, hi, theta, weights,
              stf="gauss_deriv", rel_step=1e-4, noise_rel=1e-3, sigma=None,
              per_receiver=False, keep_nominal=False, keep_J=False, stream=None,
              jacobian="fd"):
    """Returns a dict of device tensors: H1, dkl, eig, status (and sigma)."""
    dev = torch.device("cuda", ctx.device)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    S = theta.shape[0]
    R = len(receivers)
    g = tuple(grid)
    if sigma is None:
        sigma = ctx.noise_sigma_peak(g, medium, 0.5 * (np.asarray(lo) + np.asarray(hi)),
                                     noise_rel, stf, stream)
    H1 = torch.empty((S, R, 7, 7) if per_receiver else (S, 7, 7), dtype=torch.float64,
                     device=dev)
    status = torch.empty(S, dtype=torch.int32, device=dev)
    nominal = ([torch.empty((g[4] + 1, R, 2), dtype=torch.float32, device=dev)
                for _ in range(S)] if keep_nominal else None)
    J = ([torch.empty((g[4] + 1, R, 2, 7), dtype=torch.float64, device=dev)
          for _ in range(S)] if keep_J else None)
    if jacobian == "fd":
        ctx.jacobian_fd([g] * S, [medium] * S, theta, [receivers] * S, sigma, H1,
                        rel_step=rel_step, stf=stf, per_receiver=per_receiver,
                        nominal=nominal, J=J, status=status, stream=stream)
    elif jacobian == "sensitivity":
        ctx.jacobian_sensitivity([g] * S, [medium] * S, theta, [receivers] * S, sigma, H1,
                                 stf=stf, per_receiver=per_receiver, nominal=nominal, J=J,
                                 status=status, stream=stream)
    else:
        raise ValueError(f"jacobian must be 'fd' or 'sensitivity', not {jacobian!r}")
    out = {"sigma": sigma, "H1": H1, "status": status}
    if nominal is not None:
        out["nominal"] = nominal
    if J is not None:
        out["J"] = J
    prior = eigseis.make_prior(lo, hi)
    if not per_receiver:
        dkl = torch.empty(S, dtype=torch.float64, device=dev)
        logdet = torch.empty(S, dtype=torch.float64, device=dev)
        eig = torch.empty(1, dtype=torch.float64, device=dev)
        st2 = torch.empty(S, dtype=torch.int32, device=dev)
        ctx.laplace_eig(H1, prior, weights, dkl, eig, theta=theta, logdet=logdet,
                        status=st2, stream=stream)
        out.update(dkl=dkl, eig=eig, logdet=logdet, chol_status=st2)
    return out
